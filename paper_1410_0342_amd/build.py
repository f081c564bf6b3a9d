"""Build libglrm.so for gfx950 with hipcc (every source, every call)."""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build", "glrm")
LIB = os.path.join(HERE, "libglrm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# (source, extra flags, object name): dense_prec.hip is built once per precision
SOURCES = [("glrm_api.cpp", [], "glrm_api"), ("common.hip", [], "common"), ("dense.hip", [], "dense"),
           ("coo.hip", [], "coo"),
           ("impute.hip", [], "impute"), ("linalg.hip", [], "linalg"), ("smallmat.cpp", [], "smallmat"),
           ("proxprox.hip", [], "proxprox")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-pragma-unroll-threshold=1000000",
         "-I" + os.path.join(ROOT, "include")]


def dense_prec_flags(prec, lks):
    """Flags of the dense instances of one precision and loss set (0: the
    quadratic loss everywhere, 1: a per-column loss table).  FP32 keeps
    matrix-core results and accumulators in VGPRs where they fit: fewer
    AGPR<->VGPR copies, and its row pass runs 4 % faster (the bf16 forms run
    slower that way).  The bf16 forms' quadratic instances use the iterative
    ILP scheduler: their row pass runs 1.7 % faster, while the loss-table
    instances run slower with it."""
    extra = []
    if prec == 0:
        extra = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
    elif lks == 0:
        extra = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]
    return ["-DGLRM_PREC=%d" % prec, "-DGLRM_LKS=%d" % lks] + extra


SOURCES += [("dense_prec.hip", dense_prec_flags(p, l), "dense_prec%d_%d" % (p, l)) for p in (0, 1, 3) for l in (0, 1)]


def _compile(item):
    src, extra, name = item
    out = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, err))
    return out


def build(jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
