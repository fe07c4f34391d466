"""Build the debug library libsllg_ldscheck.so in-tree: the sources and
flags of libsllg.so with SLLG_LDS_CHECK defined, so that the streamed
full-width-row kernel tags every LDS slot with the plane it stands for and
checks the tag of each slot it reads (a mismatch sets a status bit that
sllg_sync reports).  Only tests load it; the product is libsllg.so."""
from __future__ import annotations

import os
import subprocess
import sys

from . import build_lib

LIB = os.path.join(build_lib.HERE, "libsllg_ldscheck.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [build_lib.HIPCC, *build_lib.FLAGS, "-DSLLG_LDS_CHECK", "-o", tmp, build_lib.SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops' is not a recognized" not in l]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building libsllg_ldscheck.so")
    if verbose and msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
