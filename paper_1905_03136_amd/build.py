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
import re
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
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]

# headers every unit includes; the C ABI header only the hand-written units
HEADERS = [os.path.join(CSRC, h) for h in ("tsg_device.hpp", "tsg_kernels.hpp", "tsg_registry.hpp")]
ABI_HEADER = os.path.join(ROOT, "include", "tsgemm.h")
TUNE_LIB = os.path.join(HERE, "libtsgemm_tune.so")
# builds of other variant sets (the autotuner's libraries): generated sources
# and objects under <repository>/_build/<tag>/, out of the package
TAGGED = os.path.join(ROOT, "_build")


def build_dirs(tag):
    """(generated sources, objects) of the build called ``tag`` ("" = the product)."""
    if not tag:
        return GEN, OBJ
    t = tag.lstrip("_")
    return os.path.join(TAGGED, t, "gen"), os.path.join(TAGGED, t, "obj")


def tagged_lib(tag):
    """Path of a named autotuning library (``tune build --tag``)."""
    return os.path.join(TAGGED, "libtsgemm_%s.so" % tag.lstrip("_"))


def _stale(obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


SPILLS = ".spills"  # per generated unit: mangled names of its kernels that spill to scratch


def _spilled(remarks):
    """Kernels with a non-zero scratch size in hipcc's resource-usage remarks."""
    out, cur = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and cur and int(m.group(1)) > 0:
            out.append(cur)
    return out


RESOURCES = ".res"  # per generated unit: register use of its kernels (JSON)


def _resources(remarks):
    """{mangled kernel name: {"vgpr", "agpr", "scratch", "occupancy"}} from
    hipcc's resource-usage remarks."""
    out, cur = {}, None
    keys = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
            "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds"}
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        for k, name in keys.items():
            m = re.search(re.escape(k) + r": (\d+)", line)
            if m and cur:
                out[cur][name] = int(m.group(1))
    return out


def _compile(src, obj, extra, resource=False):
    flags = ["-Rpass-analysis=kernel-resource-usage"] if resource else []
    cmd = [HIPCC, *CFLAGS, *extra, *flags, "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stdout[-6000:]))
    if resource:
        with open(obj + SPILLS + ".tmp", "w") as f:
            f.write("".join(k + "\n" for k in _spilled(r.stdout)))
        os.replace(obj + SPILLS + ".tmp", obj + SPILLS)
        import json
        with open(obj + RESOURCES + ".tmp", "w") as f:
            json.dump(_resources(r.stdout), f)
        os.replace(obj + RESOURCES + ".tmp", obj + RESOURCES)
    os.replace(obj + ".tmp", obj)
    return src


def variant_resources(variants, tag="_tune"):
    """{variant name: register use} of the compiled units of a build (the
    tuning library by default), from the per-unit resource records."""
    import json
    from paper_1905_03136_amd import codegen
    mangled = {}
    for f in glob.glob(os.path.join(build_dirs(tag)[1], "*" + RESOURCES)):
        with open(f) as fh:
            mangled.update(json.load(fh))
    if not mangled:
        return {}
    keys = list(mangled)
    r = subprocess.run(["c++filt"], input="\n".join(keys), stdout=subprocess.PIPE, text=True, check=True)
    by_sym = {}
    for k, d in zip(keys, r.stdout.splitlines()):
        by_sym[d.split("(")[0]] = mangled[k]
    out = {}
    for v in variants:
        sym = "void " + codegen.template_of(v)
        if sym in by_sym:
            out[codegen.variant_name(v)] = by_sym[sym]
    return out


def _spilled_variants(objs, variants):
    """Names of the variants whose kernel spills registers to scratch memory
    (from the units' resource-usage records)."""
    from paper_1905_03136_amd import codegen
    mangled = []
    for o in objs:
        if os.path.exists(o + SPILLS):
            with open(o + SPILLS) as f:
                mangled += [l.strip() for l in f if l.strip()]
    if not mangled:
        return set()
    r = subprocess.run(["c++filt"], input="\n".join(mangled), stdout=subprocess.PIPE, text=True, check=True)
    names = r.stdout.splitlines()
    out = set()
    for v in variants:
        sym = "void " + codegen.template_of(v) + "("
        if any(n.startswith(sym) for n in names):
            out.add(codegen.variant_name(v))
    return out


def generate(widths=None, variants=None, gen_dir=GEN):
    sys.path.insert(0, ROOT)
    from paper_1905_03136_amd import codegen
    if variants is None:
        variants = codegen.all_variants(widths, os.path.join(HERE, "tuned.json"))
    return codegen.emit(gen_dir, variants, batched=codegen.tuned_batched(os.path.join(HERE, "tuned.json"))), variants


def build(widths=None, jobs=None, extra_flags=(), verbose=True, variants=None, lib_path=LIB, tag=""):
    """Generate and compile.  ``variants`` replaces the product's variant set
    (the autotuner builds all candidates this way into its own library,
    objects and generated sources kept apart by ``tag``)."""
    gen_dir, obj_dir = build_dirs(tag)
    srcs, variants = generate(widths, variants, gen_dir)
    table = os.path.join(gen_dir, "tsg_table.hip")
    units = [s for s in srcs if s != table]
    srcs = units + [os.path.join(CSRC, "tsg_runtime.hip"), os.path.join(CSRC, "tsg_stream.hip"),
                    os.path.join(CSRC, "tsg_batched.hip")]
    OBJD = obj_dir
    os.makedirs(OBJD, exist_ok=True)
    obj_of = {s: os.path.join(OBJD, os.path.basename(s) + ".o") for s in srcs + [table]}
    keep = set(obj_of.values())
    for o in glob.glob(os.path.join(OBJD, "*.o")):
        if o not in keep:
            os.remove(o)
    jobs = jobs or min(8, os.cpu_count() or 1)
    # objects built with other flags are stale (the flags are kept beside them)
    stamp = os.path.join(OBJD, "flags.txt")
    flags = " ".join([HIPCC] + CFLAGS + list(extra_flags))
    same_flags = os.path.exists(stamp) and open(stamp).read() == flags

    def compile_all(sources, what):
        todo = [(s, obj_of[s]) for s in sources
                if not same_flags or _stale(obj_of[s], [s] + HEADERS + ([] if s in units else [ABI_HEADER]))
                or (s in units and not (os.path.exists(obj_of[s] + SPILLS) and
                                        os.path.exists(obj_of[s] + RESOURCES)))]
        if not todo:
            return
        if verbose:
            print("[build] compiling %d of %d %s for %s (%d variants), %d jobs"
                  % (len(todo), len(sources), what, ARCH, len(variants), jobs), flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            for done in ex.map(lambda so: _compile(so[0], so[1], list(extra_flags), so[0] in units), todo):
                if verbose:
                    print("[build]   %s" % os.path.relpath(done, ROOT), flush=True)

    # Generated units first; a variant whose kernel spills registers to
    # scratch memory is left out of the registry (its launches would be slow,
    # and spilled code is not trusted), then the table is compiled.
    compile_all(srcs, "units")
    spilled = _spilled_variants([obj_of[s] for s in units], variants)
    if spilled:
        print("[build] %d variant(s) spill registers and are left out of the registry: %s"
              % (len(spilled), ", ".join(sorted(spilled))), flush=True)
        from paper_1905_03136_amd import codegen
        codegen.emit(gen_dir, variants, exclude=spilled,
                     batched=codegen.tuned_batched(os.path.join(HERE, "tuned.json")))
    compile_all([table], "registry table")
    with open(stamp, "w") as f:
        f.write(flags)
    objs = [obj_of[s] for s in srcs] + [obj_of[table]]
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
