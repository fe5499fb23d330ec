"""Build the HIP library (gfx950) into paper_2001_10986_amd/libdd.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
LIB = os.path.join(PKG, "libdd.so")
SOURCES = ["dd_kernels.hip", "dd_runtime.hip", "dd_cert.hip", "dd_single.hip", "mlp_kernels.hip",
           "mlp_runtime.hip", "dd_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def _torch_lib_dir():
    """Directory of the HIP runtime that PyTorch loads; the library links the
    same one so that device pointers and streams are shared with torch."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return None
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def build(verbose: bool = False, jobs: int = 2) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tl = _torch_lib_dir()
    if tl:
        # plain link against the runtime torch loads (one HIP runtime per process)
        cmd = ["g++", "-shared", "-o", LIB + ".tmp", *objs, f"-L{tl}", "-l:libamdhip64.so",
               f"-Wl,-rpath,{tl}", "-Wl,--disable-new-dtags"]
    else:
        cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
