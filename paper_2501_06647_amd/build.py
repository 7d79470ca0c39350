"""Build libtucket.so in-tree with hipcc for gfx950.

Every translation unit is compiled to an object file in parallel (the six
stitch-kernel instantiations are separate units of tk_stitch_inst.hip), then
the objects are linked into one shared library.  Always recompiles.
"""

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["csrc/tk_kernels.hip", "csrc/tk_capi.hip", "csrc/tk_batch.hip", "csrc/tk_serve.hip", "csrc/tk_tail.hip", "csrc/tk_stream.hip"]
STITCH_SOURCE = "csrc/tk_stitch_inst.hip"
STITCH_INSTANCES = [(64, 4), (128, 4), (256, 4), (64, 7), (128, 7), (256, 7)]
HEADERS = ["csrc/tk_common.hpp", "csrc/tk_device.hpp", "csrc/tk_internal.hpp", "csrc/tk_host.hpp",
           "csrc/tk_stitch.hpp"]
OUT = os.path.join(HERE, "libtucket.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-pthread",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _units(src_dir, obj_dir):
    units = [(os.path.join(src_dir, s), os.path.join(obj_dir, os.path.basename(s)[:-4] + ".o"), []) for s in SOURCES]
    for ntt, pm in STITCH_INSTANCES:
        units.append((os.path.join(src_dir, STITCH_SOURCE), os.path.join(obj_dir, "tk_stitch_%d_%d.o" % (ntt, pm)),
                      ["-DTK_NTT=%d" % ntt, "-DTK_PM=%d" % pm]))
    return units


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l]
    return proc.returncode, lines


def build(verbose: bool = False, jobs: int = 0, src_dir: str = HERE, obj_dir: str = OBJ_DIR,
          out: str = OUT) -> str:
    """Compile and link; src_dir holds the csrc/ tree (default: this
    package's), objects go to obj_dir and the library to out."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(obj_dir, exist_ok=True)
    units = _units(src_dir, obj_dir)
    cmds = [[hipcc] + FLAGS + extra + ["-c", src, "-o", obj] for src, obj, extra in units]
    workers = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_run, cmds))
    for cmd, (rc, lines) in zip(cmds, results):
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + "\n".join(lines))
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", out + ".tmp"] + [o for _, o, _ in units]
    if verbose:
        print(" ".join(link), flush=True)
    rc, lines = _run(link)
    if rc != 0:
        raise RuntimeError("link failed:\n" + "\n".join(lines))
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
