"""Builds the host-code sanitizer driver (sanitize_driver.cpp) against the
library's sources compiled with AddressSanitizer and UndefinedBehaviorSanitizer
on their host code only (``-Xarch_host`` before every sanitizer flag; device
code is compiled exactly as in the library build).

    python tests/native/build_sanitized.py [-v]

The executable lands in tests/native/_build/sanitize_driver; its "cpu" mode
runs without a device, its "gpu" mode needs one.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1409_8186_amd import build as libbuild  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]


OUT = os.path.join(HERE, "_build")
DRIVER = os.path.join(OUT, "sanitize_driver")


def inputs() -> list[str]:
    """Every file the driver is built from."""
    return (libbuild.sources() + [os.path.join(HERE, "sanitize_driver.cpp"), __file__,
                                  os.path.join(ROOT, "include", "mudiff.h")]
            + [os.path.join(libbuild.CSRC, f) for f in os.listdir(libbuild.CSRC)
               if f.endswith(".h")])


def stale() -> bool:
    """True when the driver is missing or older than one of its inputs."""
    if not os.path.exists(DRIVER):
        return True
    t = os.path.getmtime(DRIVER)
    return any(os.path.getmtime(f) > t for f in inputs())


def build(verbose: bool = False) -> str:
    """Compiles every library source and the driver, links the driver; returns its path."""
    out = OUT
    os.makedirs(out, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(src: str) -> str:
        obj = os.path.join(out, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        cmd = [libbuild.HIPCC, *libbuild.FLAGS, *SAN, *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    srcs = libbuild.sources() + [os.path.join(HERE, "sanitize_driver.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = DRIVER + ".tmp"
    cmd = [libbuild.HIPCC, f"--offload-arch={libbuild.ARCH}", *SAN, "-o", exe, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(exe, DRIVER)
    return DRIVER


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
