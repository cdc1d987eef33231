"""Build libtsgemm.so in-tree for gfx950.

Runs the code generator, compiles every generated unit and the runtime with
hipcc (in parallel, skipping objects that are newer than their sources and
headers) and links the shared library next to this file.  No GPU is needed:
hipcc cross-compiles for gfx950.

    python -m paper_1905_03136_amd.build [--graded-only] [--jobs N]
"""
import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtsgemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # keep the compiler from forming packed FP32 instructions (not used here anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    "-I" + os.path.join(ROOT, "include"),
]

HEADERS = [os.path.join(CSRC, h) for h in ("tsg_device.hpp", "tsg_kernels.hpp", "tsg_registry.hpp")] + \
    [os.path.join(ROOT, "include", "tsgemm.h")]
TUNE_LIB = os.path.join(HERE, "libtsgemm_tune.so")


def _stale(obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, obj, extra):
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stdout[-6000:]))
    os.replace(obj + ".tmp", obj)
    return src


def generate(widths=None, variants=None, gen_dir=GEN):
    sys.path.insert(0, ROOT)
    from paper_1905_03136_amd import codegen
    if variants is None:
        variants = codegen.all_variants(widths, os.path.join(HERE, "tuned.json"))
    return codegen.emit(gen_dir, variants), variants


def build(widths=None, jobs=None, extra_flags=(), verbose=True, variants=None, lib_path=LIB, tag=""):
    """Generate and compile.  ``variants`` replaces the product's variant set
    (the autotuner builds all candidates this way into its own library,
    objects and generated sources kept apart by ``tag``)."""
    gen_dir = GEN + tag
    obj_dir = OBJ + tag
    srcs, variants = generate(widths, variants, gen_dir)
    srcs = list(srcs) + [os.path.join(CSRC, "tsg_runtime.hip"), os.path.join(CSRC, "tsg_stream.hip"),
                        os.path.join(CSRC, "tsg_batched.hip")]
    OBJD = obj_dir
    os.makedirs(OBJD, exist_ok=True)
    objs = []
    todo = []
    for s in srcs:
        o = os.path.join(OBJD, os.path.basename(s) + ".o")
        objs.append(o)
        if _stale(o, [s] + HEADERS + [os.path.abspath(__file__)]):
            todo.append((s, o))
    for o in glob.glob(os.path.join(OBJD, "*.o")):
        if o not in objs:
            os.remove(o)
    jobs = jobs or min(8, os.cpu_count() or 1)
    if todo:
        if verbose:
            print("[build] compiling %d of %d units for %s (%d variants), %d jobs"
                  % (len(todo), len(srcs), ARCH, len(variants), jobs), flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            for done in ex.map(lambda so: _compile(so[0], so[1], list(extra_flags)), todo):
                if verbose:
                    print("[build]   %s" % os.path.relpath(done, ROOT), flush=True)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", lib_path + ".tmp", *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stdout[-6000:])
    os.replace(lib_path + ".tmp", lib_path)
    if verbose:
        print("[build] wrote %s" % os.path.relpath(lib_path, ROOT), flush=True)
    return lib_path


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graded-only", action="store_true",
                    help="pre-generate only the sweep widths (faster build; other widths use run-time-width variants)")
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args(argv)
    widths = None
    if a.graded_only:
        from paper_1905_03136_amd import codegen
        widths = codegen.GRADED
    build(widths, a.jobs)


if __name__ == "__main__":
    main()
