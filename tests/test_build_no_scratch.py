"""Every kernel of the library compiles for gfx950 without private (scratch)
memory: a spill or a dynamically indexed local array would put per-lane
arrays in scratch, which costs a memory round trip per access."""
import glob
import re
import tempfile

from paper_2412_00578_amd.csrc import build


def test_no_kernel_uses_scratch():
    with tempfile.TemporaryDirectory() as d:
        build.dump_asm(d)
        bad = []
        for path in sorted(glob.glob(f"{d}/*.s")):
            kernel = None
            for line in open(path):
                m = re.match(r"\s*\.amdhsa_kernel\s+(\S+)", line)
                if m:
                    kernel = m.group(1)
                m = re.match(r"\s*\.amdhsa_private_segment_fixed_size\s+(\d+)", line)
                if m and int(m.group(1)) != 0:
                    bad.append((path.rsplit("/", 1)[-1], kernel, int(m.group(1))))
        assert not bad, bad
