"""Register use of the streaming kernels, read from the gfx950 assembly
(CPU only: hipcc cross-compiles).  The multi-step kernels keep several rows
of populations in registers and run two or three wavefronts per SIMD; a
kernel that spills would both slow down many times over and, where a spill
lands inside a lane-divergent region, keep the inactive lanes' values only
in registers the spill code does not restore.  So every kernel lbm_step
launches by default must compile without scratch memory, at the
wavefronts per SIMD its launch bounds ask for."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2211_03160_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isa", "stream_kernels.hip")

# kernel name fragment -> least wavefronts per SIMD
EXPECT = {
    "stream_kernelINS_7StorageINS_3E32ES2_fEELi4ELb1ELi5ELi0E": 2,
    "stream_kernelINS_7StorageINS_3E32ES2_fEELi4ELb0ELi5ELi0E": 2,
    "stream_kernelINS_7StorageINS_3E16ES2_fEELi4ELb1ELi3ELi0E": 3,
    "stream_kernelINS_7StorageINS_4EB16ES2_fEELi4ELb1ELi4ELi0E": 2,
    "stream_kernelINS_7StorageINS_3E16ENS_3E32EfEELi4ELb1ELi4ELi0E": 2,
    "batch_stream_kernelINS_7StorageINS_3E32ES2_fEELi8ELb1ELi5ELi0E": 2,
    "step_kernelILi2ENS_7StorageINS_3E32ES2_fEEEE": 4,
    "step_kernelILi3ENS_7StorageINS_3E32ES2_fEEEE": 4,
    "stream3_kernelINS_7StorageINS_3E32ES2_fEEEE": 2,
}


@pytest.mark.timeout(600)
def test_default_stream_kernels_do_not_spill(tmp_path):
    if not os.path.exists(build.HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = tmp_path / "stream_kernels.s"
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([build.HIPCC] + flags + ["--cuda-device-only", "-S", "-o", str(out), SRC],
                   check=True, capture_output=True)
    text = out.read_text().splitlines()
    found = {}
    cur = None
    for i, line in enumerate(text):
        m = re.match(r"^(_ZN3lbm\w+):", line)
        if m:
            cur = m.group(1)
        if line.startswith("; ScratchSize:") and cur:
            occ = next(int(l.split(":")[1]) for l in text[i:i + 20] if l.startswith("; Occupancy:"))
            found[cur] = (int(line.split(":")[1]), occ)
    for frag, waves in EXPECT.items():
        hits = [(k, v) for k, v in found.items() if frag in k]
        assert len(hits) == 1, (frag, list(found))
        name, (scratch, occ) = hits[0]
        assert scratch == 0, f"{name}: {scratch} bytes of scratch"
        assert occ >= waves, f"{name}: {occ} wavefronts per SIMD, expected >= {waves}"
