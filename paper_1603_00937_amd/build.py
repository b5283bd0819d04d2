"""Compiles the HIP sources of libgb for gfx950 into paper_1603_00937_amd/libgb.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["api.hip", "scan.hip", "graph.hip", "partition.hip", "mlpart.hip", "sp2.hip"]
# the rate probes: compiled on their own with the matrix cores' VGPR form, so that a loop of
# independent accumulations keeps its accumulators in place (the default form moves them
# between register files on every iteration)
PROBE_SOURCES = ["peak.hip"]
PROBE_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
LIB = os.path.join(HERE, "libgb.so")


def hipcc_flags():
    return [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result", "-Wno-unused-function",
    ]


def source_hash() -> str:
    """SHA-256 of the library sources (the tag of its autotuning tables)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(HERE, "csrc"))):
        h.update(name.encode())
        h.update(open(os.path.join(HERE, "csrc", name), "rb").read())
    h.update(open(os.path.join(HERE, "..", "include", "gb.h"), "rb").read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel; the rate probes with their own flags),
    then link libgb.so."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = LIB + ".tmp"
    sha = f'-DGB_SOURCE_SHA="{source_hash()}"'
    flags = [f for f in hipcc_flags() if f != "-shared"]
    jobs = [(n, []) for n in SOURCES] + [(n, PROBE_FLAGS) for n in PROBE_SOURCES]
    objs = [os.path.join(HERE, n + ".o") for n, _ in jobs]

    def compile_one(job):
        (name, extra), obj = job
        cmd = ["/opt/rocm/bin/hipcc", *flags, *extra, sha, "-c",
               os.path.join(HERE, "csrc", name), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return name, subprocess.run(cmd, capture_output=True, text=True)

    try:
        with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            for name, r in ex.map(compile_one, zip(jobs, objs)):
                if r.returncode != 0:
                    sys.stderr.write(r.stdout + r.stderr)
                    raise RuntimeError(f"hipcc failed compiling {name}")
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
               "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("linking libgb.so failed")
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    # every symbol must resolve at load time (a kernel whose launch stub the host pass
    # dropped shows up as an undefined symbol here, not as a compile error)
    chk = subprocess.run(
        [sys.executable, "-c", "import ctypes, sys; ctypes.CDLL(sys.argv[1], mode=2)", tmp],
        capture_output=True, text=True)
    if chk.returncode != 0:
        sys.stderr.write(chk.stderr)
        raise RuntimeError("libgb.so has unresolved symbols")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
