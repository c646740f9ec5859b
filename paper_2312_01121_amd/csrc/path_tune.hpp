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
    {4, 1, 227, 1, 0, 0},   // small
    {4, 1, 320, 2, 4, 0},   // resident
    {4, 1, 448, 2, 8, 8},   // resident
    {4, 1, 640, 3, 0, 0},   // stream
    {4, 1, 884, 2, 8, 8},   // resident
    {4, 1, 1140, 3, 0, 0},   // stream
    {4, 1, 1408, 2, 8, 8},   // resident
    {4, 1, 1792, 2, 8, 8},   // resident
    {4, 1, 2304, 2, 8, 8},   // resident
    {4, 1, 2816, 3, 0, 0},   // stream
    {4, 1, 1073741824, 3, 0, 0},   // stream
    {8, 0, 24, 1, 0, 0},   // small
    {8, 0, 40, 1, 0, 0},   // small
    {8, 0, 56, 1, 0, 0},   // small
    {8, 0, 72, 1, 0, 0},   // small
    {8, 0, 88, 1, 0, 0},   // small
    {8, 0, 112, 1, 0, 0},   // small
    {8, 0, 134, 2, 8, 0},   // resident
    {8, 0, 166, 2, 8, 0},   // resident
    {8, 0, 224, 2, 8, 0},   // resident
    {8, 0, 320, 2, 8, 0},   // resident
    {8, 0, 448, 2, 4, 4},   // resident
    {8, 0, 640, 2, 4, 4},   // resident
    {8, 0, 884, 2, 4, 4},   // resident
    {8, 0, 1140, 2, 4, 0},   // resident
    {8, 0, 1408, 2, 8, 8},   // resident
    {8, 0, 1792, 2, 8, 8},   // resident
    {8, 0, 1073741824, 2, 8, 8},   // resident
    {8, 1, 24, 1, 0, 0},   // small
    {8, 1, 40, 1, 0, 0},   // small
    {8, 1, 56, 1, 0, 0},   // small
    {8, 1, 72, 1, 0, 0},   // small
    {8, 1, 88, 1, 0, 0},   // small
    {8, 1, 112, 1, 0, 0},   // small
    {8, 1, 134, 2, 4, 0},   // resident
    {8, 1, 166, 2, 4, 0},   // resident
    {8, 1, 224, 2, 4, 0},   // resident
    {8, 1, 320, 2, 4, 0},   // resident
    {8, 1, 448, 2, 4, 0},   // resident
    {8, 1, 640, 2, 4, 0},   // resident
    {8, 1, 884, 2, 4, 4},   // resident
    {8, 1, 1140, 2, 4, 0},   // resident
    {8, 1, 1408, 2, 8, 0},   // resident
    {8, 1, 1792, 2, 8, 8},   // resident
    {8, 1, 1073741824, 3, 0, 0},   // stream
};

// Measured (dtype/coupling/n): {path or resident_wavesxrows: us per RK4 step}
// {"f32/x/1000": {"resident_16x0": 14.02, "resident_16x16": 12.54, "resident_4x0": 14.33, "resident_4x4": 14.26, "resident_8x0": 14.93, "resident_8x16": 15.98, "resident_8x8": 11.88, "stream": 17.01}, "f32/x/128": {"resident_16x0": 9.6, "resident_16x16": 8.05, "resident_4x0": 11.75, "resident_4x4": 9.97, "resident_8x0": 12.06, "resident_8x16": 13.03, "resident_8x8": 9.95, "small": 6.83, "stream": 15.39}, "f32/x/1280": {"resident_16x0": 15.07, "resident_16x16": 12.12, "resident_4x0": 20.89, "resident_4x4": 16.76, "resident_8x0": 17.57, "resident_8x16": 16.36, "resident_8x8": 12.82, "stream": 18.75}, "f32/x/1536": {"resident_16x0": 15.42, "resident_16x16": 12.87, "resident_4x0": 21.76, "resident_4x4": 17.25, "resident_8x0": 16.8, "resident_8x16": 17.26, "resident_8x8": 13.77, "stream": 18.69}, "f32/x/16": {"resident_16x0": 6.78, "resident_16x16": 7.66, "resident_4x0": 8.49, "resident_4x4": 8.92, "resident_8x0": 8.45, "resident_8x16": 11.95, "resident_8x8": 9.32, "small": 2.03, "stream": 14.48}, "f32/x/160": {"resident_16x0": 10.54, "resident_16x16": 8.29, "resident_4x0": 12.27, "resident_4x4": 10.18, "resident_8x0": 12.51, "resident_8x16": 13.42, "resident_8x8": 10.17, "small": 14.43, "stream": 15.34}, "f32/x/199": {"resident_16x0": 11.21, "resident_16x16": 8.54, "resident_4x0": 13.59, "resident_4x4": 10.69, "resident_8x0": 13.81, "resident_8x16": 13.29, "resident_8x8": 10.19, "small": 9.71, "stream": 15.19}, "f32/x/2048": {"resident_16x0": 16.58, "resident_16x16": 14.01, "resident_4x0": 22.08, "resident_4x4": 18.32, "resident_8x0": 14.98, "resident_8x16": 18.98, "resident_8x8": 14.97, "stream": 23.87}, "f32/x/256": {"resident_16x0": 11.82, "resident_16x16": 8.4, "resident_4x0": 13.08, "resident_4x4": 10.89, "resident_8x0": 13.25, "resident_8x16": 13.08, "resident_8x8": 10.1, "stream": 15.5}, "f32/x/2560": {"resident_16x0": 18.58, "resident_4x0": 31.69, "resident_4x4": 21.65, "resident_8x0": 24.29, "stream": 26.04}, "f32/x/3072": {"resident_16x0": 19.93, "resident_4x0": 34.02, "resident_8x0": 26.24, "stream": 30.95}, "f32/x/32": {"resident_16x0": 7.39, "resident_16x16": 7.7, "resident_4x0": 9.27, "resident_4x4": 8.89, "resident_8x0": 9.3, "resident_8x16": 12.49, "resident_8x8": 9.87, "small": 2.3, "stream": 14.62}, "f32/x/384": {"resident_16x0": 10.83, "resident_16x16": 8.7, "resident_4x0": 13.26, "resident_4x4": 11.68, "resident_8x0": 13.73, "resident_8x16": 13.67, "resident_8x8": 10.59, "stream": 16.78}, "f32/x/512": {"resident_16x0": 11.62, "resident_16x16": 9.09, "resident_4x0": 13.99, "resident_4x4": 12.68, "resident_8x0": 14.39, "resident_8x16": 14.4, "resident_8x8": 11.09, "stream": 15.62}, "f32/x/64": {"resident_16x0": 8.0, "resident_16x16": 7.68, "resident_4x0": 10.57, "resident_4x4": 9.64, "resident_8x0": 10.85, "resident_8x16": 11.7, "resident_8x8": 10.34, "small": 3.65, "stream": 15.08}, "f32/x/768": {"resident_16x0": 13.71, "resident_16x16": 9.91, "resident_4x0": 16.55, "resident_4x4": 13.93, "resident_8x0": 16.34, "resident_8x16": 14.59, "resident_8x8": 11.48, "stream": 17.13}, "f32/x/96": {"resident_16x0": 8.86, "resident_16x16": 8.22, "resident_4x0": 11.5, "resident_4x4": 9.86, "resident_8x0": 11.82, "resident_8x16": 13.49, "resident_8x8": 10.53, "small": 4.96, "stream": 15.2}, "f32/xyz/1000": {"resident_16x0": 27.57, "resident_16x16": 24.08, "resident_4x0": 19.9, "resident_4x4": 19.92, "resident_8x0": 20.75, "resident_8x16": 24.78, "resident_8x8": 19.25, "stream": 19.13}, "f32/xyz/128": {"resident_16x0": 15.98, "resident_16x16": 17.36, "resident_4x0": 14.96, "resident_4x4": 15.6, "resident_8x0": 14.97, "resident_8x16": 20.14, "resident_8x8": 15.78, "small": 8.55, "stream": 16.74}, "f32/xyz/1280": {"resident_16x0": 28.73, "resident_16x16": 25.6, "resident_4x0": 32.37, "resident_4x4": 27.03, "resident_8x0": 23.79, "resident_8x16": 25.98, "resident_8x8": 20.11, "stream": 21.31}, "f32/xyz/1536": {"resident_16x0": 29.42, "resident_16x16": 27.32, "resident_4x0": 32.9, "resident_4x4": 28.52, "resident_8x0": 22.62, "resident_8x16": 27.36, "resident_8x8": 20.91, "stream": 21.36}, "f32/xyz/16": {"resident_16x0": 12.91, "resident_16x16": 15.73, "resident_4x0": 13.47, "resident_4x4": 14.43, "resident_8x0": 13.64, "resident_8x16": 18.38, "resident_8x8": 15.22, "small": 2.36, "stream": 14.8}, "f32/xyz/160": {"resident_16x0": 17.35, "resident_16x16": 17.62, "resident_4x0": 15.4, "resident_4x4": 16.14, "resident_8x0": 15.74, "resident_8x16": 20.18, "resident_8x8": 16.07, "small": 17.93, "stream": 16.64}, "f32/xyz/199": {"resident_16x0": 18.45, "resident_16x16": 18.18, "resident_4x0": 16.65, "resident_4x4": 16.63, "resident_8x0": 17.07, "resident_8x16": 20.56, "resident_8x8": 16.5, "small": 15.69, "stream": 16.53}, "f32/xyz/2048": {"resident_16x0": 32.1, "resident_16x16": 30.29, "resident_4x0": 35.26, "resident_4x4": 30.86, "resident_8x0": 22.41, "resident_8x16": 29.77, "resident_8x8": 22.4, "stream": 25.83}, "f32/xyz/256": {"resident_16x0": 18.01, "resident_16x16": 18.01, "resident_4x0": 15.8, "resident_4x4": 16.25, "resident_8x0": 16.07, "resident_8x16": 19.66, "resident_8x8": 15.92, "stream": 16.75}, "f32/xyz/2560": {"resident_16x0": 32.86, "resident_4x0": 51.23, "resident_8x0": 37.4, "stream": 30.44}, "f32/xyz/3072": {"stream": 37.47}, "f32/xyz/32": {"resident_16x0": 13.02, "resident_16x16": 15.82, "resident_4x0": 14.11, "resident_4x4": 14.59, "resident_8x0": 13.76, "resident_8x16": 18.97, "resident_8x8": 15.71, "small": 2.65, "stream": 15.91}, "f32/xyz/384": {"resident_16x0": 19.96, "resident_16x16": 19.04, "resident_4x0": 17.11, "resident_4x4": 17.61, "resident_8x0": 17.57, "resident_8x16": 21.0, "resident_8x8": 16.94, "stream": 18.73}, "f32/xyz/512": {"resident_16x0": 21.65, "resident_16x16": 19.78, "resident_4x0": 17.58, "resident_4x4": 17.82, "resident_8x0": 18.25, "resident_8x16": 21.72, "resident_8x8": 17.26, "stream": 17.12}, "f32/xyz/64": {"resident_16x0": 13.07, "resident_16x16": 15.77, "resident_4x0": 14.39, "resident_4x4": 15.55, "resident_8x0": 14.39, "resident_8x16": 17.34, "resident_8x8": 16.31, "small": 4.51, "stream": 16.57}, "f32/xyz/768": {"resident_16x0": 25.69, "resident_16x16": 21.25, "resident_4x0": 20.69, "resident_4x4": 19.04, "resident_8x0": 21.63, "resident_8x16": 22.99, "resident_8x8": 18.35, "stream": 19.16}, "f32/xyz/96": {"resident_16x0": 15.74, "resident_16x16": 17.58, "resident_4x0": 14.97, "resident_4x4": 15.8, "resident_8x0": 15.01, "resident_8x16": 20.67, "resident_8x8": 16.54, "small": 5.97, "stream": 16.56}, "f64/x/1000": {"resident_16x0": 17.34, "resident_16x16": 21.83, "resident_4x0": 14.03, "resident_4x4": 14.04, "resident_8x0": 15.13, "resident_8x16": 25.57, "resident_8x8": 16.62, "stream": 21.25}, "f64/x/128": {"resident_16x0": 10.51, "resident_16x16": 13.68, "resident_4x0": 10.31, "resident_4x4": 10.69, "resident_8x0": 10.21, "resident_8x16": 18.41, "resident_8x8": 13.14, "small": 11.66, "stream": 17.39}, "f64/x/1280": {"resident_16x0": 19.08, "resident_4x0": 23.67, "resident_4x4": 20.9, "resident_8x0": 18.33, "resident_8x8": 17.65, "stream": 26.4}, "f64/x/140": {"resident_16x0": 11.5, "resident_16x16": 14.27, "resident_4x0": 10.48, "resident_4x4": 10.82, "resident_8x0": 10.43, "resident_8x16": 18.92, "resident_8x8": 13.43, "small": 15.06, "stream": 18.55}, "f64/x/1536": {"resident_16x0": 20.83, "resident_4x0": 27.21, "resident_4x4": 22.7, "resident_8x0": 19.21, "resident_8x8": 19.2, "stream": 26.05}, "f64/x/16": {"resident_16x0": 8.85, "resident_16x16": 12.5, "resident_4x0": 9.85, "resident_4x4": 10.57, "resident_8x0": 9.68, "resident_8x16": 16.77, "resident_8x8": 12.54, "small": 2.84, "stream": 15.91}, "f64/x/192": {"resident_16x0": 11.63, "resident_16x16": 14.54, "resident_4x0": 10.83, "resident_4x4": 11.12, "resident_8x0": 10.75, "resident_8x16": 18.81, "resident_8x8": 13.45, "stream": 18.47}, "f64/x/2048": {"resident_16x0": 24.59, "resident_4x0": 30.65, "resident_8x0": 23.74, "resident_8x8": 23.73, "stream": 31.02}, "f64/x/256": {"resident_16x0": 12.35, "resident_16x16": 14.61, "resident_4x0": 10.91, "resident_4x4": 11.01, "resident_8x0": 10.89, "resident_8x16": 19.02, "resident_8x8": 13.34, "stream": 18.62}, "f64/x/32": {"resident_16x0": 9.12, "resident_16x16": 12.26, "resident_4x0": 10.18, "resident_4x4": 11.19, "resident_8x0": 10.12, "resident_8x16": 15.74, "resident_8x8": 11.29, "small": 3.36, "stream": 17.04}, "f64/x/384": {"resident_16x0": 13.34, "resident_16x16": 15.75, "resident_4x0": 11.76, "resident_4x4": 11.44, "resident_8x0": 11.88, "resident_8x16": 20.05, "resident_8x8": 13.84, "stream": 19.96}, "f64/x/48": {"resident_16x0": 9.15, "resident_16x16": 13.21, "resident_4x0": 9.86, "resident_4x4": 10.9, "resident_8x0": 9.99, "resident_8x16": 17.55, "resident_8x8": 13.1, "small": 4.57, "stream": 17.32}, "f64/x/512": {"resident_16x0": 14.16, "resident_16x16": 16.67, "resident_4x0": 11.99, "resident_4x4": 11.76, "resident_8x0": 12.15, "resident_8x16": 20.83, "resident_8x8": 14.01, "stream": 18.52}, "f64/x/64": {"resident_16x0": 9.42, "resident_16x16": 12.34, "resident_4x0": 9.99, "resident_4x4": 10.62, "resident_8x0": 9.83, "resident_8x16": 15.87, "resident_8x8": 13.06, "small": 6.77, "stream": 17.4}, "f64/x/768": {"resident_16x0": 17.24, "resident_16x16": 19.55, "resident_4x0": 13.94, "resident_4x4": 12.81, "resident_8x0": 14.93, "resident_8x16": 23.46, "resident_8x8": 15.26, "stream": 21.17}, "f64/x/80": {"resident_16x0": 10.06, "resident_16x16": 13.89, "resident_4x0": 10.61, "resident_4x4": 11.08, "resident_8x0": 10.5, "resident_8x16": 18.57, "resident_8x8": 13.72, "small": 7.26, "stream": 17.21}, "f64/x/96": {"resident_16x0": 10.51, "resident_16x16": 13.96, "resident_4x0": 10.48, "resident_4x4": 10.88, "resident_8x0": 10.36, "resident_8x16": 18.62, "resident_8x8": 13.55, "small": 8.02, "stream": 17.33}, "f64/xyz/1000": {"resident_16x0": 34.82, "resident_16x16": 48.62, "resident_4x0": 25.97, "resident_4x4": 26.05, "resident_8x0": 30.45, "resident_8x16": 53.94, "resident_8x8": 33.88, "stream": 31.72}, "f64/xyz/128": {"resident_16x0": 18.89, "resident_16x16": 28.67, "resident_4x0": 17.48, "resident_4x4": 18.15, "resident_8x0": 17.67, "resident_8x16": 32.18, "resident_8x8": 22.27, "small": 24.79, "stream": 20.32}, "f64/xyz/1280": {"resident_16x0": 38.51, "resident_4x0": 48.48, "resident_4x4": 44.73, "resident_8x0": 36.79, "resident_8x8": 36.8, "stream": 38.58}, "f64/xyz/140": {"resident_16x0": 19.76, "resident_16x16": 29.49, "resident_4x0": 18.21, "resident_4x4": 18.87, "resident_8x0": 18.56, "resident_8x16": 34.17, "resident_8x8": 23.53, "small": 34.25, "stream": 22.02}, "f64/xyz/1536": {"resident_16x0": 43.03, "resident_4x0": 54.59, "resident_8x0": 40.19, "resident_8x8": 39.97, "stream": 41.3}, "f64/xyz/16": {"resident_16x0": 17.73, "resident_16x16": 27.13, "resident_4x0": 17.25, "resident_4x4": 18.17, "resident_8x0": 17.45, "resident_8x16": 30.25, "resident_8x8": 21.74, "small": 4.32, "stream": 19.27}, "f64/xyz/192": {"resident_16x0": 19.85, "resident_16x16": 29.53, "resident_4x0": 18.31, "resident_4x4": 18.79, "resident_8x0": 18.7, "resident_8x16": 33.61, "resident_8x8": 23.31, "stream": 21.8}, "f64/xyz/2048": {"stream": 54.63}, "f64/xyz/256": {"resident_16x0": 20.56, "resident_16x16": 30.4, "resident_4x0": 18.6, "resident_4x4": 19.2, "resident_8x0": 18.98, "resident_8x16": 34.53, "resident_8x8": 23.59, "stream": 21.87}, "f64/xyz/32": {"resident_16x0": 17.87, "resident_16x16": 27.11, "resident_4x0": 17.9, "resident_4x4": 18.67, "resident_8x0": 17.99, "resident_8x16": 29.07, "resident_8x8": 20.55, "small": 5.14, "stream": 20.04}, "f64/xyz/384": {"resident_16x0": 23.9, "resident_16x16": 32.98, "resident_4x0": 20.32, "resident_4x4": 20.42, "resident_8x0": 21.35, "resident_8x16": 37.98, "resident_8x8": 25.74, "stream": 23.91}, "f64/xyz/48": {"resident_16x0": 17.83, "resident_16x16": 27.81, "resident_4x0": 17.5, "resident_4x4": 18.55, "resident_8x0": 17.92, "resident_8x16": 32.12, "resident_8x8": 22.57, "small": 8.04, "stream": 20.11}, "f64/xyz/512": {"resident_16x0": 25.43, "resident_16x16": 35.55, "resident_4x0": 21.3, "resident_4x4": 21.39, "resident_8x0": 22.44, "resident_8x16": 40.54, "resident_8x8": 26.98, "stream": 25.13}, "f64/xyz/64": {"resident_16x0": 17.7, "resident_16x16": 27.17, "resident_4x0": 17.47, "resident_4x4": 18.09, "resident_8x0": 17.58, "resident_8x16": 29.65, "resident_8x8": 22.41, "small": 12.58, "stream": 20.35}, "f64/xyz/768": {"resident_16x0": 29.44, "resident_16x16": 40.93, "resident_4x0": 23.78, "resident_4x4": 23.72, "resident_8x0": 25.25, "resident_8x16": 46.85, "resident_8x8": 30.35, "stream": 28.77}, "f64/xyz/80": {"resident_16x0": 19.61, "resident_16x16": 29.33, "resident_4x0": 18.58, "resident_4x4": 18.92, "resident_8x0": 18.44, "resident_8x16": 34.04, "resident_8x8": 23.16, "small": 14.43, "stream": 20.16}, "f64/xyz/96": {"resident_16x0": 19.58, "resident_16x16": 29.27, "resident_4x0": 18.18, "resident_4x4": 18.46, "resident_8x0": 18.25, "resident_8x16": 33.95, "resident_8x8": 22.97, "small": 16.32, "stream": 20.28}}

}  // namespace sto
