"""mps_amplitudes_noalloc (the entry point for callers that cannot allocate) against
mps_amplitudes through the C ABI: the same amplitude kernels read their tables
from a fixed device array instead of the engine's staging areas, so the results
must agree bit for bit.  Two calls in a row, the second on a smaller state with
fewer bitstrings (the array keeps the first call's contents), FP64 and dd; a
request beyond the array's size is refused with MPS_ERANGE before any device
work."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def state(B, n, chi, depth, seed, dd):
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    d = B.MPS(n, chi, 1e-12, prec)
    d.apply_gates([g for layer in W.brickwork(n, depth, seed) for g in layer])
    return d


def same(a, b):
    return np.array_equal(a.view(np.float64), b.view(np.float64))


@pytest.mark.parametrize("dd", [False, True])
def test_noalloc_matches_amplitudes(B, dd):
    # first call: 14 qubits, 300 bitstrings; second: 9 qubits, 17 bitstrings
    for n, chi, depth, seed, count in ((14, 24, 8, 71, 300), (9, 8, 5, 72, 17)):
        print(f"noalloc: n={n} chi={chi} depth={depth} seed={seed} count={count} dd={dd}", flush=True)
        d = state(B, n, chi, depth, seed, dd)
        bits = W.bitstrings(n, count, seed + 100)
        if dd:
            rh, rl = d.amplitudes(bits, dd=True)
            gh, gl = d.amplitudes(bits, dd=True, noalloc=True)
            assert same(rh, gh) and same(rl, gl)
            assert np.max(np.abs(gh)) > 0
        else:
            ref = d.amplitudes(bits)
            got = d.amplitudes(bits, noalloc=True)
            assert same(ref, got)
            assert np.max(np.abs(got)) > 0
        d.close()


def test_noalloc_rejects_oversize(B):
    d = B.MPS(60, 4, 0.0)
    bits = np.zeros((60000, 60), dtype=np.uint8)  # 60000 x 60 bits + results > 4 MiB
    with pytest.raises(B.MPSError) as ei:
        d.amplitudes(bits, noalloc=True)
    assert ei.value.code == B.MPS_ERANGE
    # the handle still answers afterwards, on both paths
    one = np.zeros((1, 60), dtype=np.uint8)
    assert d.amplitudes(one, noalloc=True)[0] == 1.0
    assert d.amplitudes(one)[0] == 1.0
    d.close()
