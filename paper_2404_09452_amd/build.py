"""Compile the HIP sources of the DF-J/K library for gfx950 into libdfjk.so."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdfjk.so")
SOURCES = ["host.hip", "integrals.hip", "linalg.hip", "jk.hip", "syrk_mixed.hip", "export.hip", "direct.hip",
           "align.hip", "bound.hip", "syrk_f64.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + SRC]


def _compile(name):
    src = os.path.join(SRC, name)
    obj = os.path.join(OBJ, name + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (name, "\n".join(msgs)))
    return obj, msgs


def _stale(name):
    """True if the object is older than its source or any header."""
    obj = os.path.join(OBJ, name + ".o")
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(SRC, name)] + [os.path.join(SRC, h) for h in os.listdir(SRC) if h.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "dfjk.h"))
    return any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def build(verbose=False, jobs=None, incremental=False):
    """Compile every source (or, with incremental=True, only stale ones) and link."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    todo = [s for s in SOURCES if not incremental or _stale(s)]
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, todo))
    results += [(os.path.join(OBJ, s + ".o"), []) for s in SOURCES if s not in todo]
    if verbose:
        for _, msgs in results:
            for m in msgs:
                print(m)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
