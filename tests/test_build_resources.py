"""Per-lane scratch memory of every kernel in the lane, wide-shard and
run-time parameter sources, as the compiler reports it when it builds them
with the library's own flags.  These kernels fully unroll their walk over a
lane's k-mers so that every per-k-mer array is indexed by constants and held
in registers; when an instantiation exceeds the compiler's unroll budget its
arrays go to scratch memory, and it runs 5-20 times slower while producing
the same bits, which no parity test notices.  A few spilled registers (tens of
bytes) are normal; a walk in scratch takes kilobytes."""

import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2606_24417_amd import build as B

SOURCES = ["kernels_rolling.hip", "kernels_wide.hip", "kernels_param.hip"]
MAX_SCRATCH_BYTES_PER_LANE = 128


def _resources(src):
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC", "-pthread")]
    cmd = ([B.hipcc()] + flags + B.SOURCE_FLAGS.get(src, []) +
           ["-I" + os.path.join(B.ROOT, "include"), "-I" + B.CSRC, "--offload-device-only", "-c", "-o", os.devnull,
            os.path.join(B.CSRC, src), "-Rpass-analysis=kernel-resource-usage"])
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert res.returncode == 0, res.stdout[-2000:]
    kernels, cur = {}, None
    for line in res.stdout.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and cur is not None:
            kernels[cur] = int(m.group(1))
    return src, kernels


@pytest.mark.skipif(shutil.which(B.hipcc()) is None and not os.path.exists(B.hipcc()), reason="no hipcc")
def test_kernels_keep_their_walk_in_registers():
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        found = dict(ex.map(_resources, SOURCES))
    for src, kernels in found.items():
        assert kernels, "no kernel resource report for %s" % src
        over = {k: v for k, v in kernels.items() if v > MAX_SCRATCH_BYTES_PER_LANE}
        assert not over, "%s: kernels using more than %d bytes of scratch per lane: %s" % (
            src, MAX_SCRATCH_BYTES_PER_LANE, over)
    # every compiled lane kernel set is covered (six sets: insert and query)
    assert sum("query_lane_kernel" in k for k in found["kernels_rolling.hip"]) >= 12
