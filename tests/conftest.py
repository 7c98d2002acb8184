import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_terminal_summary(terminalreporter):
    helpers = sys.modules.get("gpu_helpers")
    rows = getattr(helpers, "EXCLUSIONS", None)
    if not rows:
        return
    tr = terminalreporter
    tr.section("FP32 cost parity near collision-indicator switches")
    tot = sum(r[4] for r in rows)
    near = sum(r[2] for r in rows)
    flips = sum(r[3] for r in rows)
    tr.write_line(f"{tot} samples in {len(rows)} comparisons: {tot - near} matched to the tolerance; {near} within "
                  f"the band of a switch, checked modulo whole indicator terms ({flips} of them flipped)")
    for test, what, n_near, n_flip, n in rows:
        if n_near:
            tr.write_line(f"  {test} {what}: {n_near} of {n} near a switch, {n_flip} flipped")
