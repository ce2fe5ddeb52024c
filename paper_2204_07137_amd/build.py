"""Build step: compiles the HIP sources into the in-tree shared library libshacsim.so.

    python -m paper_2204_07137_amd.build                   # libshacsim.so
    python -m paper_2204_07137_amd.build --phase-profile   # libshacsim_phase.so (phase marks)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libshacsim.so")
LIB_PHASE = os.path.join(HERE, "libshacsim_phase.so")
# the window kernels are split over several units (one precision's full layouts, compact
# layouts and group kernels) that compile in parallel
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels_f32_group_fwd.hip", "kernels_f32_group_adj.hip", "kernels_f32.hip",
                                                  "kernels_f32_compact.hip", "kernels_f64.hip", "kernels_f64_group_fwd.hip",
                                                  "kernels_f64_group_adj.hip", "shacsim_abi.hip", "learn.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("sim_types.h", "sim_math.h", "sim_dynamics.h", "sim_task.h", "sim_gemm.h", "sim_learn.h",
                                                 "sim_kernels.h", "sim_unit_f32.h", "sim_unit_f64.h")] + [
    os.path.join(ROOT, "include", "shacsim.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SHACSIM_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # floating-point contraction decided per source expression, so that a substep
    # recomputed inside the adjoint is bitwise identical to the forward's
    "-ffp-contract=on",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=False, phase_profile=False):
    """Compiles the library; with phase_profile the window kernels carry the phase marks
    (-DSIM_PHASE_PROFILE) and the result is libshacsim_phase.so."""
    lib = LIB_PHASE if phase_profile else LIB
    objdir = os.path.join(HERE, "_build_phase" if phase_profile else "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + (["-DSIM_PHASE_PROFILE"] if phase_profile else []) + [
            "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    failed = False
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed compiling libshacsim sources")
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", lib + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed linking {os.path.basename(lib)}")
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    out = build(verbose=True, phase_profile="--phase-profile" in sys.argv[1:])
    print("built", out)
