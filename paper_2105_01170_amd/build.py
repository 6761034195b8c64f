"""Compile the HIP sources of the t-SVDM library for gfx950 into libtsvdm.so.

Each file under csrc/ is compiled to an object by its own hipcc invocation (in
parallel), then the objects are linked into a shared library with a plain C
interface (include/tsvdm.h).  Packed-FP32 instruction selection is disabled
(-packed-fp32-ops) for all device code.  Per-file options:

  batched.hip: -amdgpu-mfma-vgpr-form.  The Gram kernel carries up to ten FP64
  MFMA accumulators across its column loop; with the default register classes
  they are copied between accumulation and vector registers on every
  iteration (about 160 extra moves per step); the vector-register form keeps
  them in place and needs fewer registers (162 instead of 244).
"""
import glob
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtsvdm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]
PER_FILE = {"batched.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    tmpdir = tempfile.mkdtemp(prefix="tsvdm_build_")
    try:
        srcs = sources()
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC] + COMMON + PER_FILE.get(os.path.basename(s), []) + ["-c", s, "-o", o]
                for s, o in zip(srcs, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs, verbose)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
