"""Build the HIP library for gfx950 in-tree (no JIT cache): ``_build/libmorph_hip.so``."""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB_NAME = "libmorph_hip.so"
SOURCES = ("k_fused_u8.hip", "k_fused_u16.hip", "k_tile.hip", "k_stream.hip", "k_stream_coop.hip", "k_wave.hip",
           "k_rows.hip", "k_wave_tall_u8.hip", "k_wave_tall_u16.hip", "morph_launch.hip", "morph_api.hip", "morph_transpose.hip",
           "morph_openclose.hip", "k_oc_u8.hip", "k_oc_u16.hip", "morph_static.hip")
ARCH = os.environ.get("MORPH_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _flags():
    return [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
            "-Rpass-analysis=kernel-resource-usage"]


_SCRATCH = re.compile(r"ScratchSize \[bytes/lane\]: (\d+)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 feature and says so; the
    # resource-usage remarks are read below, not printed; keep real errors
    lines = [ln for ln in res.stdout.splitlines()
             if "packed-fp32-ops" not in ln and "kernel-resource-usage" not in ln]
    if res.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed (%d)" % res.returncode)
    # a kernel whose registers spill to scratch memory runs many times slower with
    # no other sign: refuse to build one
    spills = [int(m) for m in _SCRATCH.findall(res.stdout) if int(m) > 0]
    if spills:
        raise RuntimeError("a kernel of %s uses %d bytes of scratch per lane (register "
                           "spills)" % (cmd[cmd.index("-c") + 1] if "-c" in cmd else "?",
                                        max(spills)))
    warnings = [ln for ln in lines if "warning:" in ln]
    if verbose and warnings:
        print("\n".join(warnings))


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the library."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OUT_DIR, exist_ok=True)
    out = os.path.join(OUT_DIR, LIB_NAME)
    tag = ".tmp%d" % os.getpid()
    objs = [os.path.join(OUT_DIR, os.path.splitext(s)[0] + tag + ".o") for s in SOURCES]
    cmds = [_flags() + ["-x", "hip", "-c", os.path.join(CSRC, s), "-o", o]
            for s, o in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(len(cmds)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = out + tag
        _run([hipcc(), "--offload-arch=" + ARCH, "-fPIC", "-shared"] + objs + ["-o", tmp],
             verbose)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
