"""Compile the HIP library libmortar.so for gfx950 (hipcc, in-tree).

Every translation unit is compiled in parallel, then linked.  Packed FP32 instructions
are disabled for all device code (the compiler would otherwise form them from plain
float arithmetic).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libmortar.so")
ARCH = os.environ.get("MORTAR_ARCH", "gfx950")

SOURCES = ["mortar_capi.hip", "k_topology.hip", "k_flux_f32.hip", "k_flux_f64.hip",
           "k_flux_wide_f32.hip", "k_flux_hyb_f32.hip", "k_lift.hip",
           "k_flux_rd_f32.hip", "k_flux_rd_f64.hip", "k_flux_rd_bf16.hip",
           "k_flux_rd_fp16.hip", "k_flux_rd_batch_f32.hip",
           "k_flux_mfma_f32.hip", "k_flux_mfma_f64.hip", "k_flux_batch_f32.hip",
           "k_flux_batch_f64.hip", "k_flux_hi_f32.hip", "k_flux_hi_f64.hip", "k_lift_hi.hip",
           "k_lift_rd_f32.hip"]

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wall", "-Wno-unused-function"]


# The register-direct and hybrid kernels keep matrix-core results in ordinary VGPRs
# (they feed the vector units and LDS directly); not used for the FP64 unit, on which
# this compiler option makes the compiler itself crash.
EXTRA = {s: ["-mllvm", "-amdgpu-mfma-vgpr-form"]
         for s in ("k_flux_rd_f32.hip", "k_flux_rd_bf16.hip", "k_flux_rd_fp16.hip",
                   "k_flux_rd_batch_f32.hip", "k_flux_hyb_f32.hip", "k_lift_rd_f32.hip")}


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-c", *CFLAGS, *EXTRA.get(src, []), "-o", obj, os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj, r.stderr


# The DGSEM solver that embeds the operator in a whole scheme (its own library; it calls
# nothing in libmortar.so, the driver passes device buffers between the two).
DG_SOURCES = ["dg_embed.hip"]
DG_OUT = os.path.join(HERE, "libdgembed.so")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES) + len(DG_SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES + DG_SOURCES))
    dg_objs = [o for o, _ in results[len(SOURCES):]]
    results = results[:len(SOURCES)]
    tmp = DG_OUT + ".tmp"
    subprocess.run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *dg_objs], check=True)
    os.replace(tmp, DG_OUT)
    if verbose:
        for _, err in results:
            if err.strip():
                print(err)
    objs = [o for o, _ in results]
    tmp = OUT + ".tmp"
    subprocess.run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
