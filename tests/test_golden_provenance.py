"""The stored oracle samples of the 128^3 hot-spot event (FP64 and reduced
state) come from the oracle step as it is now and from the event's current
seeded input: each file records the SHA-256 of the oracle source its run
depended on and of the initial energy densities.  A change to either fails
here on the CPU, before the GPU parity tests would refuse the files."""
import hashlib
import os

import numpy as np
import pytest

from paper_1608_06577_amd import inputs as I
from tests.golden import make_hotspot_golden as mk_fp64
from tests.golden import make_reduced_golden as mk_red

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,mk", [("hotspot_128_fp64.npz", mk_fp64), ("hotspot_128_reduced_fp64.npz", mk_red)])
def test_samples_match_the_current_oracle_and_input(name, mk):
    gold = np.load(os.path.join(GOLDEN, name))
    assert np.array_equal(gold["oracle_sha"], mk.oracle_sha()), \
        "the oracle step changed since %s was written: run its tests/golden/make_*.py" % name
    e = I.workload_hotspot().prims.e
    sha = hashlib.sha256(np.ascontiguousarray(e).tobytes()).digest()
    assert np.array_equal(np.frombuffer(sha, np.uint8), gold["input_sha"])
