"""micsa_read_c4_static (no device allocation, a static scratch array per
device) against micsa_read_c4 (which allocates its buffers), through the C
ABI: equal on two calls in a row, the second on a smaller lattice (the
array keeps the first call's contents), on both layouts; a lattice beyond
the array's limit is refused with ERANGE."""
import numpy as np
import pytest

from paper_2506_16240_amd import micsa as M

pytestmark = pytest.mark.gpu


def _swept(shape, layout=M.LAYOUT_BYTE, seed=5, n=6):
    g = M.Lattice(*shape, seed, layout=layout)
    g.set_schedule(M.Schedule(M.SCHED_CONST, 0.9, 0.9, n, 3))
    g.sweep(M.ALGO_MICSA, n)
    return g


def test_c4_static_equals_c4_on_consecutive_calls():
    big = _swept((64, 32, 16, 3, 4))  # several samples and pairs, ragged rows of 32 words
    small = _swept((16, 8, 8, 1, 2))
    bit = _swept((32, 8, 8, 70, 2), layout=M.LAYOUT_BITPLANE)
    for g in (big, small, bit, big):
        want = g.c4_sums()
        got = g.c4_sums_static()
        assert np.array_equal(got, want)
        # a second call in a row on the same lattice
        assert np.array_equal(g.c4_sums_static(), want)
    for g in (big, small, bit):
        g.close()


def test_c4_static_refuses_what_does_not_fit():
    g = M.Lattice(8, 8, 8, 5000, 2, 1)  # 5000 samples x 3 axes x 5 distances of count slots
    with pytest.raises(M.MicsaError) as e:
        g.c4_sums_static()
    assert e.value.status == M.ERANGE
    assert g.c4_sums().shape == (5000, 3, 5)  # the allocating call still serves it
    g.close()
