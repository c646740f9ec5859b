"""Register budget of the built kernels, read from the code object metadata
of libsto_reservoir.so (no GPU): no kernel spills to scratch memory except
the instances listed below, and every 1,024-thread kernel fits 128 vector
registers per lane (four waves per SIMD), which the 16-wave launch shapes
need."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2312_01121_amd", "libsto_reservoir.so")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

# Instances that spill, off the hot path or at its edge: the readout's
# Cholesky panel (once per fit), and the multi-stream reverse with isotropic
# coupling, two row tiles and KREG = 32 (N = 513-1,024).
SPILL_ALLOWED = ("k_bpanel", "k_multi_revILi32ELb1ELi2E")


def kernels(tmp):
    """Metadata (name, registers, scratch, workgroup size) of every kernel."""
    fat = os.path.join(tmp, "fatbin.bin")
    subprocess.run([f"{LLVM}/llvm-objcopy", "--dump-section", f".hip_fatbin={fat}", LIB,
                    os.path.join(tmp, "discard.so")], check=True)
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(b"__CLANG_OFFLOAD_BUNDLE__"), data)]
    out = []
    for j, s in enumerate(starts):
        chunk = os.path.join(tmp, f"b{j}.bin")
        code = os.path.join(tmp, f"d{j}.co")
        with open(chunk, "wb") as fh:
            fh.write(data[s:starts[j + 1] if j + 1 < len(starts) else len(data)])
        subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={chunk}",
                        f"--targets={TARGET}", f"--output={code}"], check=True)
        notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", code], capture_output=True, text=True,
                               check=True).stdout
        cur = {}
        for line in notes.splitlines():
            m = re.match(r"\s*(-\s+)?\.(\w+):\s*(\S+)", line)
            if not m:
                continue
            if m.group(2) == "agpr_count" and m.group(1):
                if "name" in cur:
                    out.append(cur)
                cur = {}
            cur[m.group(2)] = m.group(3)
        if "name" in cur:
            out.append(cur)
    return [k for k in out if "vgpr_count" in k]


@pytest.fixture(scope="module")
def meta(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    if not all(shutil.which(os.path.join(LLVM, t)) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")):
        pytest.skip("LLVM tools not found")
    ks = kernels(str(tmp_path_factory.mktemp("codeobj")))
    assert len(ks) > 100
    return ks


def test_no_unexpected_spills(meta):
    spills = [k["name"] for k in meta if int(k.get("private_segment_fixed_size", 0)) > 0]
    unexpected = [n for n in spills if not any(a in n for a in SPILL_ALLOWED)]
    assert not unexpected, unexpected


def test_sixteen_wave_kernels_fit_128_registers(meta):
    big = [(k["name"], k["vgpr_count"], k.get("agpr_count")) for k in meta
           if int(k.get("max_flat_workgroup_size", 0)) == 1024
           and int(k["vgpr_count"]) + int(k.get("agpr_count", 0)) > 128]
    assert not big, big


def test_hot_kernels_are_present(meta):
    names = " ".join(k["name"] for k in meta)
    for kernel in ("k_stage", "k_small", "k_resident", "k_multi", "k_sweep_stage", "k_adj_stage"):
        assert kernel in names, kernel
