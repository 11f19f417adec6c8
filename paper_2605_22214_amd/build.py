"""Build the HIP library libnflbm.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2605_22214_amd.build [--changed]  (or build() from
Python); --changed recompiles only the units older than a source or header.
Objects go to _build/ at the repository root; the shared library is written
next to this file so that it ships with the package tree.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnflbm.so")
ARCH = os.environ.get("NFLBM_OFFLOAD_ARCH", "gfx950")

# Device-code flags: gfx950 only; packed FP32 instructions are kept out of the
# generated code (the compiler would otherwise form them from float code).
# No implicit contraction of a*b + c: the kernels spell their fused
# multiply-adds as fma(), so every instantiation of a kernel body (single or
# batch launch, either storage form of g) rounds identically.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off"]
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
          "-Wall", "-Wno-unused-function"]

# Translation units: (source, object, is_device_code, extra defines)
# kernels.hip is compiled once per storage precision, lattice and group of
# component counts (each unit registers its launchers when the library
# loads), so that the units build in parallel; NFLBM_COMPONENTS (e.g. "5")
# restricts a development build to those N.
_NC_GROUPS = {0: [(2, 4), (5, 8)], 1: [(2, 3), (4, 4), (5, 5), (6, 6), (7, 7), (8, 8)]}


def _kernel_units():
    only = os.environ.get("NFLBM_COMPONENTS")
    only = {int(v) for v in only.split(",")} if only else None
    out = []
    for st, name in ((0, "f64"), (1, "f32"), (2, "f16s")):
        for lat in (0, 1):
            for lo, hi in _NC_GROUPS[lat]:
                if only is not None:
                    sel = sorted(n for n in only if lo <= n <= hi)
                    if not sel:
                        continue
                    lo, hi = sel[0], sel[-1]
                out.append(("kernels.hip", f"kernels_{name}_l{lat}_n{lo}{hi}.o", True,
                            [f"-DNFLBM_UNIT_STORE={st}", f"-DNFLBM_UNIT_LAT={lat}",
                             f"-DNFLBM_UNIT_NC_LO={lo}", f"-DNFLBM_UNIT_NC_HI={hi}"]))
    return out


UNITS = [
    ("coeffs.cpp", "coeffs.o", False, []),
    ("api.cpp", "api.o", False, []),
] + _kernel_units() + [
    ("kernels.hip", "kernels_common.o", True, ["-DNFLBM_UNIT_STORE=-1"]),
    ("mobility.hip", "mobility.o", True, []),
    ("outflow.hip", "outflow.o", True, []),
    ("noalloc.hip", "noalloc.o", True, []),
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def _compile(unit):
    src, obj, device, defs = unit
    cmd = [hipcc()] + COMMON + defs
    if device:
        cmd += ["-x", "hip", f"--offload-arch={ARCH}"] + DEVICE_FLAGS
    else:
        # host-only C++ that calls the HIP runtime API
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    t = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj, time.time() - t, res.stderr


def _stale(unit):
    """True if the unit's object is missing or older than its source or any
    header it may include (every header of csrc/ and include/)."""
    obj = os.path.join(BUILD, unit[1])
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, unit[0])]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    inc = os.path.join(ROOT, "include")
    deps += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose=True, jobs=None, changed_only=False):
    """Compile every unit (changed_only: only those whose object is older
    than a source or header) and link libnflbm.so."""
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if _stale(u)] if changed_only else UNITS
    # the D3Q19 kernel units take longest: start them first
    units = sorted(units, key=lambda u: ("_l1_" not in u[1], u[1]))
    jobs = jobs or min(max(len(units), 1), os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, warn in ex.map(_compile, units):
            if verbose:
                print(f"  compiled {obj} in {dt:.1f}s", flush=True)
                w = "\n".join(l for l in warn.splitlines() if "packed-fp32-ops" not in l
                              and "not a recognized feature" not in l)
                if w.strip():
                    print(w, flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
          [os.path.join(BUILD, u[1]) for u in UNITS] + ["-L/opt/rocm/lib", "-lhipfft"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"  linked {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(changed_only="--changed" in sys.argv[1:])
    sys.exit(0)
