"""Build libfpn.so (HIP kernels for gfx950 + C ABI) in-tree.

Usage: python paper_2106_08040_amd/build.py [-v]
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfpn.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _runtime_dir():
    """Directory of the libamdhip64.so the Python process uses (PyTorch's), else /opt/rocm/lib."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return "/opt/rocm/lib"
# packed FP32 VALU instructions are disabled for all device code
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def _fresh(cmd, newest_header):
    """True when the object a compile step writes is newer than its source and every header."""
    src = cmd[cmd.index("-c") + 1]
    obj = cmd[cmd.index("-o") + 1]
    return os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(src), newest_header)


def build(jobs=8, verbose=False, out=None, build_dir=None, extra=(), incremental=False):
    """Compile every source and link libfpn.so.  incremental=True (development only) skips objects
    that are newer than their source and all headers."""
    BUILD = build_dir or globals()["BUILD"]
    LIB = out or globals()["LIB"]
    HIP_FLAGS = [*globals()["HIP_FLAGS"], *extra]
    os.makedirs(BUILD, exist_ok=True)
    # the stepper is instantiated per Galerkin degree; split across objects to compile in parallel
    ranges = [(1, 6), (7, 10), (11, 13), (14, 15), (16, 16)]
    step_objs = [os.path.join(BUILD, f"stepper_{a}_{b}.o") for a, b in ranges]
    wide_ranges = [(17, 18), (19, 20), (21, 22), (23, 23), (24, 24)]
    wide_objs = [os.path.join(BUILD, f"stepper_wide_{a}_{b}.o") for a, b in wide_ranges]
    steps = [
        [HIPCC, *HIP_FLAGS, f"-DFPN_L_BEGIN={a}", f"-DFPN_L_END={b}", "-c", os.path.join(CSRC, "stepper.hip"),
         "-o", o] for (a, b), o in zip(ranges, step_objs)
    ] + [
        [HIPCC, *HIP_FLAGS, f"-DFPN_L_BEGIN={a}", f"-DFPN_L_END={b}", "-c", os.path.join(CSRC, "stepper_wide.hip"),
         "-o", o] for (a, b), o in zip(wide_ranges, wide_objs)
    ] + [
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(BUILD, "kernels.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "capi.hip"), "-o", os.path.join(BUILD, "capi.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "mlp.hip"), "-o", os.path.join(BUILD, "mlp.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "capi_mlp.hip"), "-o", os.path.join(BUILD, "capi_mlp.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "surrogate.hip"), "-o", os.path.join(BUILD, "surrogate.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "capi_surrogate.hip"), "-o",
         os.path.join(BUILD, "capi_surrogate.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "capi_static.hip"), "-o", os.path.join(BUILD, "capi_static.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "capi_surmodel.hip"), "-o",
         os.path.join(BUILD, "capi_surmodel.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "fit.hip"), "-o", os.path.join(BUILD, "fit.o")],
        ["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, "structure.cpp"),
         "-o", os.path.join(BUILD, "structure.o")],
        ["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, "m2_host.cpp"),
         "-o", os.path.join(BUILD, "m2_host.o")],
    ]
    if incremental:
        hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
        hdrs.append(os.path.join(HERE, "..", "include", "fpn.h"))
        newest = max(os.path.getmtime(h) for h in hdrs)
        steps = [c for c in steps if not _fresh(c, newest)]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, steps))
    if verbose:
        for o in outs:
            print(o, end="")
    tmp = LIB + ".tmp"
    # Link against the HIP runtime that PyTorch loads (NEEDED libamdhip64.so, torch's copy first on
    # the runpath) so one process never holds two HIP/HSA runtimes; /opt/rocm/lib is the fallback.
    hiplib = _runtime_dir()
    _run([CLANG, "-shared", "-fPIC", "-o", tmp, *step_objs, *wide_objs,
          os.path.join(BUILD, "kernels.o"), os.path.join(BUILD, "capi.o"), os.path.join(BUILD, "structure.o"),
          os.path.join(BUILD, "mlp.o"), os.path.join(BUILD, "capi_mlp.o"),
          os.path.join(BUILD, "surrogate.o"), os.path.join(BUILD, "capi_surrogate.o"),
          os.path.join(BUILD, "capi_static.o"), os.path.join(BUILD, "capi_surmodel.o"),
          os.path.join(BUILD, "fit.o"), os.path.join(BUILD, "m2_host.o"),
          f"-L{hiplib}", "-l:libamdhip64.so", f"-Wl,-rpath,{hiplib}:/opt/rocm/lib", "-lstdc++"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
