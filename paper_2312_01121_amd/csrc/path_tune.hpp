// Path and launch shape of a single-stream reservoir by element type,
// coupling and size, chosen by measurement.  Written by
// paper_2312_01121_amd/autotune.py --paths; entries are scanned in order and
// the first with matching element size and coupling and n <= n_max applies.
// Each measured size covers n up to the midpoint to the next; above the last
// one the entry's path holds while it can (the resident path falls back to
// the stream path where W no longer fits the CUs' LDS).
#pragma once

namespace sto {

struct PathTuneEntry {
    int elem_bytes;
    int xyz;        // 0: m^x coupling, 1: all three components
    int n_max;
    int path;       // 1 small, 2 resident, 3 stream (sto_path values)
    int waves;      // resident: waves per workgroup (4, 8 or 16)
    int rpb;        // resident: rows per workgroup (0: ceil(n / CUs))
};

// Fastest path and shape per size bucket (microseconds per RK4 step measured
// for every path and resident shape that holds the size; listed below).
constexpr PathTuneEntry kPathTune[] = {
    {4, 0, 24, 1, 0, 0},   // small
    {4, 0, 48, 1, 0, 0},   // small
    {4, 0, 80, 1, 0, 0},   // small
    {4, 0, 112, 1, 0, 0},   // small
    {4, 0, 144, 1, 0, 0},   // small
    {4, 0, 179, 2, 16, 16},   // resident
    {4, 0, 227, 2, 16, 16},   // resident
    {4, 0, 320, 2, 16, 16},   // resident
    {4, 0, 448, 2, 16, 16},   // resident
    {4, 0, 640, 2, 16, 16},   // resident
    {4, 0, 884, 2, 16, 16},   // resident
    {4, 0, 1140, 2, 8, 8},   // resident
    {4, 0, 1408, 2, 16, 16},   // resident
    {4, 0, 1792, 2, 16, 16},   // resident
    {4, 0, 2304, 2, 16, 16},   // resident
    {4, 0, 2816, 2, 16, 0},   // resident
    {4, 0, 1073741824, 2, 16, 0},   // resident
    {4, 1, 24, 1, 0, 0},   // small
    {4, 1, 48, 1, 0, 0},   // small
    {4, 1, 80, 1, 0, 0},   // small
    {4, 1, 112, 1, 0, 0},   // small
    {4, 1, 144, 1, 0, 0},   // small
    {4, 1, 179, 2, 4, 0},   // resident
    {4, 1, 227, 2, 8, 8},   // resident
    {4, 1, 320, 2, 8, 8},   // resident
    {4, 1, 448, 2, 8, 8},   // resident
    {4, 1, 640, 3, 0, 0},   // stream
    {4, 1, 884, 2, 8, 8},   // resident
    {4, 1, 1140, 3, 0, 0},   // stream
    {4, 1, 1408, 2, 8, 8},   // resident
    {4, 1, 1792, 2, 8, 8},   // resident
    {4, 1, 2304, 2, 8, 0},   // resident
    {4, 1, 2816, 3, 0, 0},   // stream
    {4, 1, 1073741824, 3, 0, 0},   // stream
    {8, 0, 24, 1, 0, 0},   // small
    {8, 0, 40, 1, 0, 0},   // small
    {8, 0, 56, 1, 0, 0},   // small
    {8, 0, 72, 1, 0, 0},   // small
    {8, 0, 88, 1, 0, 0},   // small
    {8, 0, 112, 1, 0, 0},   // small
    {8, 0, 134, 2, 4, 0},   // resident
    {8, 0, 166, 2, 4, 0},   // resident
    {8, 0, 224, 2, 4, 0},   // resident
    {8, 0, 320, 2, 4, 0},   // resident
    {8, 0, 448, 2, 4, 4},   // resident
    {8, 0, 640, 2, 4, 4},   // resident
    {8, 0, 884, 2, 4, 4},   // resident
    {8, 0, 1140, 2, 4, 4},   // resident
    {8, 0, 1408, 2, 8, 8},   // resident
    {8, 0, 1792, 2, 8, 0},   // resident
    {8, 0, 1073741824, 2, 8, 8},   // resident
    {8, 1, 24, 1, 0, 0},   // small
    {8, 1, 40, 1, 0, 0},   // small
    {8, 1, 56, 1, 0, 0},   // small
    {8, 1, 72, 1, 0, 0},   // small
    {8, 1, 88, 1, 0, 0},   // small
    {8, 1, 112, 2, 4, 0},   // resident
    {8, 1, 134, 2, 4, 0},   // resident
    {8, 1, 166, 2, 4, 0},   // resident
    {8, 1, 224, 2, 4, 0},   // resident
    {8, 1, 320, 2, 4, 0},   // resident
    {8, 1, 448, 2, 4, 0},   // resident
    {8, 1, 640, 2, 4, 0},   // resident
    {8, 1, 884, 2, 4, 0},   // resident
    {8, 1, 1140, 2, 4, 0},   // resident
    {8, 1, 1408, 2, 8, 0},   // resident
    {8, 1, 1792, 2, 8, 8},   // resident
    {8, 1, 1073741824, 3, 0, 0},   // stream
};

// Measured (dtype/coupling/n): {path or resident_wavesxrows: us per RK4 step}
// {"f32/x/1000": {"resident_16x0": 14.6, "resident_16x16": 13.55, "resident_4x0": 14.28, "resident_4x4": 14.29, "resident_8x0": 15.2, "resident_8x16": 17.24, "resident_8x8": 13.06, "stream": 17.66}, "f32/x/128": {"resident_16x0": 10.39, "resident_16x16": 8.42, "resident_4x0": 12.89, "resident_4x4": 10.2, "resident_8x0": 13.0, "resident_8x16": 14.17, "resident_8x8": 10.36, "small": 8.04, "stream": 15.92}, "f32/x/1280": {"resident_16x0": 16.08, "resident_16x16": 13.29, "resident_4x0": 22.4, "resident_4x4": 16.72, "resident_8x0": 18.59, "resident_8x16": 17.75, "resident_8x8": 14.54, "stream": 19.32}, "f32/x/1536": {"resident_16x0": 16.45, "resident_16x16": 14.3, "resident_4x0": 23.14, "resident_4x4": 17.15, "resident_8x0": 18.13, "resident_8x16": 18.6, "resident_8x8": 15.66, "stream": 19.26}, "f32/x/16": {"resident_16x0": 7.55, "resident_16x16": 8.07, "resident_4x0": 9.42, "resident_4x4": 8.63, "resident_8x0": 9.55, "resident_8x16": 12.29, "resident_8x8": 8.89, "small": 2.61, "stream": 15.4}, "f32/x/160": {"resident_16x0": 11.19, "resident_16x16": 8.52, "resident_4x0": 13.36, "resident_4x4": 10.76, "resident_8x0": 13.44, "resident_8x16": 14.63, "resident_8x8": 10.81, "small": 14.88, "stream": 16.15}, "f32/x/199": {"resident_16x0": 10.95, "resident_16x16": 9.61, "resident_4x0": 14.21, "resident_4x4": 11.23, "resident_8x0": 14.32, "resident_8x16": 14.83, "resident_8x8": 10.68, "small": 10.04, "stream": 15.98}, "f32/x/2048": {"resident_16x0": 17.64, "resident_16x16": 15.78, "resident_4x0": 23.31, "resident_4x4": 18.19, "resident_8x0": 17.09, "resident_8x16": 20.62, "resident_8x8": 17.17, "stream": 23.96}, "f32/x/256": {"resident_16x0": 11.78, "resident_16x16": 8.86, "resident_4x0": 13.89, "resident_4x4": 11.18, "resident_8x0": 14.0, "resident_8x16": 14.22, "resident_8x8": 10.66, "stream": 16.18}, "f32/x/2560": {"resident_16x0": 20.2, "resident_4x0": 34.13, "resident_4x4": 21.85, "resident_8x0": 26.14, "stream": 25.27}, "f32/x/3072": {"resident_16x0": 21.63, "resident_4x0": 35.75, "resident_8x0": 28.01, "stream": 31.77}, "f32/x/32": {"resident_16x0": 8.2, "resident_16x16": 8.07, "resident_4x0": 10.29, "resident_4x4": 9.53, "resident_8x0": 10.43, "resident_8x16": 12.37, "resident_8x8": 9.19, "small": 3.15, "stream": 15.76}, "f32/x/384": {"resident_16x0": 11.06, "resident_16x16": 9.17, "resident_4x0": 13.99, "resident_4x4": 12.1, "resident_8x0": 14.48, "resident_8x16": 14.84, "resident_8x8": 11.17, "stream": 17.57}, "f32/x/512": {"resident_16x0": 11.95, "resident_16x16": 9.57, "resident_4x0": 14.68, "resident_4x4": 12.89, "resident_8x0": 15.1, "resident_8x16": 15.55, "resident_8x8": 11.61, "stream": 16.27}, "f32/x/64": {"resident_16x0": 8.7, "resident_16x16": 8.27, "resident_4x0": 11.68, "resident_4x4": 9.98, "resident_8x0": 11.96, "resident_8x16": 13.97, "resident_8x8": 10.72, "small": 4.34, "stream": 15.65}, "f32/x/768": {"resident_16x0": 13.58, "resident_16x16": 10.43, "resident_4x0": 16.83, "resident_4x4": 13.93, "resident_8x0": 16.91, "resident_8x16": 15.85, "resident_8x8": 12.54, "stream": 17.78}, "f32/x/96": {"resident_16x0": 9.6, "resident_16x16": 8.57, "resident_4x0": 12.6, "resident_4x4": 10.41, "resident_8x0": 12.71, "resident_8x16": 14.62, "resident_8x8": 10.66, "small": 5.46, "stream": 15.77}, "f32/xyz/1000": {"resident_16x0": 27.59, "resident_16x16": 24.76, "resident_4x0": 20.99, "resident_4x4": 21.03, "resident_8x0": 21.73, "resident_8x16": 27.88, "resident_8x8": 20.51, "stream": 20.2}, "f32/xyz/128": {"resident_16x0": 16.62, "resident_16x16": 18.03, "resident_4x0": 16.29, "resident_4x4": 16.77, "resident_8x0": 16.32, "resident_8x16": 21.74, "resident_8x8": 16.71, "small": 11.93, "stream": 17.48}, "f32/xyz/1280": {"resident_16x0": 29.44, "resident_16x16": 26.88, "resident_4x0": 36.29, "resident_4x4": 28.38, "resident_8x0": 25.39, "resident_8x16": 29.36, "resident_8x8": 21.39, "stream": 22.16}, "f32/xyz/1536": {"resident_16x0": 29.91, "resident_16x16": 28.65, "resident_4x0": 37.24, "resident_4x4": 29.78, "resident_8x0": 24.5, "resident_8x16": 31.13, "resident_8x8": 22.21, "stream": 22.23}, "f32/xyz/16": {"resident_16x0": 14.09, "resident_16x16": 16.23, "resident_4x0": 14.75, "resident_4x4": 13.93, "resident_8x0": 14.77, "resident_8x16": 18.47, "resident_8x8": 14.53, "small": 3.8, "stream": 15.68}, "f32/xyz/160": {"resident_16x0": 17.92, "resident_16x16": 18.33, "resident_4x0": 16.92, "resident_4x4": 17.3, "resident_8x0": 17.07, "resident_8x16": 21.9, "resident_8x8": 17.26, "small": 20.38, "stream": 17.61}, "f32/xyz/199": {"resident_16x0": 19.05, "resident_16x16": 19.09, "resident_4x0": 18.02, "resident_4x4": 17.82, "resident_8x0": 18.49, "resident_8x16": 22.36, "resident_8x8": 17.5, "small": 18.46, "stream": 17.56}, "f32/xyz/2048": {"resident_16x0": 32.27, "resident_16x16": 32.21, "resident_4x0": 40.55, "resident_4x4": 32.03, "resident_8x0": 23.69, "resident_8x16": 34.23, "resident_8x8": 23.7, "stream": 26.64}, "f32/xyz/256": {"resident_16x0": 18.56, "resident_16x16": 18.84, "resident_4x0": 17.19, "resident_4x4": 17.33, "resident_8x0": 17.36, "resident_8x16": 21.66, "resident_8x8": 17.08, "stream": 17.65}, "f32/xyz/2560": {"resident_16x0": 33.13, "resident_4x0": 57.97, "resident_8x0": 42.97, "stream": 31.36}, "f32/xyz/3072": {"stream": 38.7}, "f32/xyz/32": {"resident_16x0": 14.34, "resident_16x16": 16.24, "resident_4x0": 15.12, "resident_4x4": 15.66, "resident_8x0": 15.0, "resident_8x16": 18.72, "resident_8x8": 14.84, "small": 4.94, "stream": 16.7}, "f32/xyz/384": {"resident_16x0": 20.37, "resident_16x16": 19.95, "resident_4x0": 18.37, "resident_4x4": 18.69, "resident_8x0": 18.8, "resident_8x16": 23.09, "resident_8x8": 18.15, "stream": 19.58}, "f32/xyz/512": {"resident_16x0": 22.02, "resident_16x16": 20.88, "resident_4x0": 18.68, "resident_4x4": 18.99, "resident_8x0": 19.45, "resident_8x16": 24.14, "resident_8x8": 18.47, "stream": 18.06}, "f32/xyz/64": {"resident_16x0": 14.93, "resident_16x16": 16.67, "resident_4x0": 15.62, "resident_4x4": 16.68, "resident_8x0": 15.58, "resident_8x16": 21.44, "resident_8x8": 17.28, "small": 6.84, "stream": 17.38}, "f32/xyz/768": {"resident_16x0": 25.83, "resident_16x16": 22.36, "resident_4x0": 21.79, "resident_4x4": 20.12, "resident_8x0": 22.65, "resident_8x16": 25.85, "resident_8x8": 19.56, "stream": 20.05}, "f32/xyz/96": {"resident_16x0": 16.4, "resident_16x16": 18.49, "resident_4x0": 16.33, "resident_4x4": 16.99, "resident_8x0": 16.29, "resident_8x16": 22.4, "resident_8x8": 17.27, "small": 8.44, "stream": 17.4}, "f64/x/1000": {"resident_16x0": 19.12, "resident_16x16": 22.71, "resident_4x0": 14.51, "resident_4x4": 14.5, "resident_8x0": 15.9, "resident_8x16": 26.6, "resident_8x8": 17.34, "stream": 21.64}, "f64/x/128": {"resident_16x0": 11.18, "resident_16x16": 13.84, "resident_4x0": 10.55, "resident_4x4": 10.97, "resident_8x0": 10.71, "resident_8x16": 18.52, "resident_8x8": 13.4, "small": 13.87, "stream": 18.06}, "f64/x/1280": {"resident_16x0": 19.68, "resident_4x0": 24.52, "resident_4x4": 20.84, "resident_8x0": 19.26, "resident_8x8": 19.01, "stream": 26.5}, "f64/x/140": {"resident_16x0": 12.12, "resident_16x16": 14.31, "resident_4x0": 10.81, "resident_4x4": 11.26, "resident_8x0": 10.95, "resident_8x16": 18.91, "resident_8x8": 13.58, "small": 17.6, "stream": 19.29}, "f64/x/1536": {"resident_16x0": 21.7, "resident_4x0": 27.63, "resident_4x4": 22.44, "resident_8x0": 20.82, "resident_8x8": 21.15, "stream": 26.2}, "f64/x/16": {"resident_16x0": 9.29, "resident_16x16": 12.35, "resident_4x0": 10.4, "resident_4x4": 9.79, "resident_8x0": 10.31, "resident_8x16": 15.93, "resident_8x8": 11.51, "small": 3.36, "stream": 16.79}, "f64/x/192": {"resident_16x0": 12.22, "resident_16x16": 14.53, "resident_4x0": 11.15, "resident_4x4": 11.51, "resident_8x0": 11.23, "resident_8x16": 19.2, "resident_8x8": 13.88, "stream": 19.29}, "f64/x/2048": {"resident_16x0": 25.47, "resident_4x0": 30.06, "resident_8x0": 25.26, "resident_8x8": 25.23, "stream": 30.99}, "f64/x/256": {"resident_16x0": 12.88, "resident_16x16": 15.03, "resident_4x0": 11.2, "resident_4x4": 11.4, "resident_8x0": 11.35, "resident_8x16": 19.18, "resident_8x8": 13.67, "stream": 19.27}, "f64/x/32": {"resident_16x0": 9.54, "resident_16x16": 13.15, "resident_4x0": 10.52, "resident_4x4": 11.42, "resident_8x0": 10.59, "resident_8x16": 17.52, "resident_8x8": 13.77, "small": 4.11, "stream": 17.68}, "f64/x/384": {"resident_16x0": 14.3, "resident_16x16": 16.27, "resident_4x0": 12.06, "resident_4x4": 11.83, "resident_8x0": 12.41, "resident_8x16": 20.37, "resident_8x8": 14.37, "stream": 20.65}, "f64/x/48": {"resident_16x0": 9.7, "resident_16x16": 12.41, "resident_4x0": 10.25, "resident_4x4": 11.39, "resident_8x0": 10.51, "resident_8x16": 15.94, "resident_8x8": 13.18, "small": 5.33, "stream": 17.9}, "f64/x/512": {"resident_16x0": 15.15, "resident_16x16": 17.22, "resident_4x0": 12.31, "resident_4x4": 12.17, "resident_8x0": 12.6, "resident_8x16": 21.11, "resident_8x8": 14.52, "stream": 19.1}, "f64/x/64": {"resident_16x0": 9.98, "resident_16x16": 13.26, "resident_4x0": 10.2, "resident_4x4": 10.87, "resident_8x0": 10.27, "resident_8x16": 17.78, "resident_8x8": 13.54, "small": 8.27, "stream": 17.92}, "f64/x/768": {"resident_16x0": 18.6, "resident_16x16": 20.1, "resident_4x0": 14.32, "resident_4x4": 13.22, "resident_8x0": 15.91, "resident_8x16": 23.67, "resident_8x8": 15.6, "stream": 21.74}, "f64/x/80": {"resident_16x0": 10.58, "resident_16x16": 14.71, "resident_4x0": 10.95, "resident_4x4": 11.52, "resident_8x0": 11.0, "resident_8x16": 19.25, "resident_8x8": 14.18, "small": 8.65, "stream": 17.79}, "f64/x/96": {"resident_16x0": 11.03, "resident_16x16": 14.28, "resident_4x0": 10.75, "resident_4x4": 11.2, "resident_8x0": 10.87, "resident_8x16": 19.02, "resident_8x8": 13.68, "small": 9.53, "stream": 17.97}, "f64/xyz/1000": {"resident_16x0": 36.75, "resident_16x16": 48.44, "resident_4x0": 26.87, "resident_4x4": 26.87, "resident_8x0": 31.72, "resident_8x16": 53.95, "resident_8x8": 34.66, "stream": 32.31}, "f64/xyz/128": {"resident_16x0": 19.37, "resident_16x16": 29.53, "resident_4x0": 17.89, "resident_4x4": 19.05, "resident_8x0": 18.08, "resident_8x16": 32.15, "resident_8x8": 22.9, "small": 28.68, "stream": 20.89}, "f64/xyz/1280": {"resident_16x0": 39.29, "resident_4x0": 49.4, "resident_4x4": 45.8, "resident_8x0": 37.5, "resident_8x8": 37.62, "stream": 39.47}, "f64/xyz/140": {"resident_16x0": 20.09, "resident_16x16": 30.4, "resident_4x0": 18.56, "resident_4x4": 19.76, "resident_8x0": 18.88, "resident_8x16": 34.18, "resident_8x8": 24.24, "small": 37.19, "stream": 22.56}, "f64/xyz/1536": {"resident_16x0": 43.62, "resident_4x0": 55.78, "resident_8x0": 41.16, "resident_8x8": 41.03, "stream": 42.25}, "f64/xyz/16": {"resident_16x0": 17.89, "resident_16x16": 27.82, "resident_4x0": 18.53, "resident_4x4": 17.72, "resident_8x0": 17.87, "resident_8x16": 29.33, "resident_8x8": 21.25, "small": 5.59, "stream": 20.03}, "f64/xyz/192": {"resident_16x0": 20.13, "resident_16x16": 30.34, "resident_4x0": 18.83, "resident_4x4": 19.88, "resident_8x0": 19.16, "resident_8x16": 33.99, "resident_8x8": 24.16, "stream": 22.34}, "f64/xyz/2048": {"stream": 55.6}, "f64/xyz/256": {"resident_16x0": 21.02, "resident_16x16": 31.39, "resident_4x0": 19.05, "resident_4x4": 20.14, "resident_8x0": 19.42, "resident_8x16": 34.76, "resident_8x8": 24.39, "stream": 22.45}, "f64/xyz/32": {"resident_16x0": 18.12, "resident_16x16": 28.59, "resident_4x0": 18.42, "resident_4x4": 19.49, "resident_8x0": 18.26, "resident_8x16": 31.23, "resident_8x8": 23.45, "small": 7.65, "stream": 20.61}, "f64/xyz/384": {"resident_16x0": 24.9, "resident_16x16": 33.48, "resident_4x0": 20.81, "resident_4x4": 21.24, "resident_8x0": 22.4, "resident_8x16": 38.4, "resident_8x8": 26.3, "stream": 24.41}, "f64/xyz/48": {"resident_16x0": 18.01, "resident_16x16": 28.03, "resident_4x0": 18.12, "resident_4x4": 19.55, "resident_8x0": 18.29, "resident_8x16": 29.53, "resident_8x8": 23.06, "small": 10.54, "stream": 20.86}, "f64/xyz/512": {"resident_16x0": 26.57, "resident_16x16": 35.77, "resident_4x0": 21.85, "resident_4x4": 22.35, "resident_8x0": 24.06, "resident_8x16": 40.83, "resident_8x8": 27.78, "stream": 25.63}, "f64/xyz/64": {"resident_16x0": 17.98, "resident_16x16": 28.58, "resident_4x0": 17.83, "resident_4x4": 18.9, "resident_8x0": 17.94, "resident_8x16": 31.73, "resident_8x8": 23.0, "small": 16.79, "stream": 20.78}, "f64/xyz/768": {"resident_16x0": 31.93, "resident_16x16": 41.03, "resident_4x0": 24.45, "resident_4x4": 24.64, "resident_8x0": 26.75, "resident_8x16": 46.82, "resident_8x8": 30.91, "stream": 29.32}, "f64/xyz/80": {"resident_16x0": 19.92, "resident_16x16": 30.38, "resident_4x0": 18.51, "resident_4x4": 20.02, "resident_8x0": 18.89, "resident_8x16": 33.72, "resident_8x8": 23.95, "small": 17.47, "stream": 20.78}, "f64/xyz/96": {"resident_16x0": 19.84, "resident_16x16": 30.22, "resident_4x0": 18.32, "resident_4x4": 19.42, "resident_8x0": 18.71, "resident_8x16": 33.83, "resident_8x8": 23.65, "small": 19.48, "stream": 20.91}}

}  // namespace sto
