"""Build libtfs.so (HIP kernels for gfx950 + host plan code) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtfs.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("tfs_kernels.hip", "tfs_adjoint.hip", "tfs_fused.hip", "tfs_ns.hip", "tfs_transport.hip",
                                                          "tfs_field.hip", "tfs_spectral.hip", "tfs_host.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off: hipcc would otherwise form them from scalar code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a multiply-add fuses only within one source expression (HIP's default also fuses across
    # statements, where the choice follows each template instance's code shape): every
    # variant of a kernel (vector width, whole waves or masked tail) rounds a point alike,
    # so results do not depend on where a point falls in a launch
    "-ffp-contract=on",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _filtered(text: str) -> str:
    return "\n".join(l for l in text.splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source to an object (in parallel), then link libtfs.so."""
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "csrc", "_" + os.path.basename(src) + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *(extra or []), *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for cmd, pr in procs:
        out = _filtered(pr.communicate()[0])
        if pr.returncode != 0:
            failed.append(f"{' '.join(cmd)}\n{out}")
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    # the transforms of the coupled step and the spectral layout: hipFFT (resolved against the copy already loaded by
    # torch when there is one, since the sonames agree)
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-L/opt/rocm/lib", "-lhipfft", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = _filtered(r.stdout + r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"link failed ({r.returncode}):\n{out}")
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
