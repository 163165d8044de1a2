"""Host checks of the tuning table and the autotuner's search space (no device):
the committed table parses under the library's rules (sections keyed by
architecture and HIP runtime version; rows of precision, largest column count,
block width 4/8/16, inner-sweep limit, QR switch), each precision's rows cover
increasing sizes, and the candidates the autotuner times are the supported ones."""
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(os.path.dirname(HERE), "paper_1111_3124_amd", "tuning.txt")


def parse(path):
    sections, cur = {}, None
    for line in open(path):
        w = line.split()
        if not w or w[0].startswith("#"):
            continue
        if w[0] == "key":
            cur = sections.setdefault(" ".join(w[1:3]), [])
            continue
        assert cur is not None, "row before any key"
        prec, nmax, bw, inner, qr = w[0], *map(int, w[1:5])
        cur.append((prec, nmax, bw, inner, qr))
    return sections


def test_committed_table_is_valid():
    sections = parse(TABLE)
    assert sections, "no section"
    for key, rows in sections.items():
        arch, ver = key.split()
        assert arch.startswith("gfx") and ver.isdigit()
        for prec in ("fp64", "dd"):
            mine = [r for r in rows if r[0] == prec]
            assert mine, (key, prec)
            sizes = [r[1] for r in mine]
            assert sizes == sorted(set(sizes))
            for _, nmax, bw, inner, qr in mine:
                assert bw in (4, 8, 16) and 1 <= inner <= 64 and qr in (0, 1) and nmax >= 1
                # QR preconditioning needs at least 64 columns; dd keeps its margin of
                # inner sweeps on small problems
                assert qr == 0 or nmax >= 64
                if prec == "dd":
                    assert inner == 12


def test_autotuner_candidates():
    pytest.importorskip("numpy")
    import importlib
    # the module imports the device binding, which needs the built library
    try:
        at = importlib.import_module("paper_1111_3124_amd.autotune")
    except (ImportError, OSError) as e:
        pytest.skip(f"library not built: {e}")
    B = at.B
    for N in (32, 64, 128, 512, 1024):
        for prec in (B.MPS_PREC_FP64, B.MPS_PREC_DD):
            cands = at.candidates(prec, N)
            assert cands and len(set(cands)) == len(cands)
            for bw, inner, qr in cands:
                assert bw in (4, 8, 16)
                assert qr in ((0, 1) if N >= 64 else (0,))
                assert inner in ((12,) if prec == B.MPS_PREC_DD else (1, 2, 4))
    # class shapes: gates on disjoint pairs whose three bonds all hold chi values
    for chi in (16, 64, 256):
        n, C, states, gates = at.layer_case(chi, 1)
        dims = [1] + [len(l) for l in states[0][1]] + [1]
        for c, g in gates:
            assert 0 <= c < C and g.k == 2
            assert dims[g.first] == dims[g.first + 1] == dims[g.first + 2] == chi
        # whole circuits of up to 12 gates: the concurrency rounded up
        assert at.CONCURRENCY[chi] <= len(gates) < at.CONCURRENCY[chi] + 12
        n3, C3, st3, g3 = at.layer_case(chi, 2, at.FEW, 3)
        assert len(g3) == at.FEW
        d3 = [1] + [len(l) for l in st3[0][1]] + [1]
        for c, g in g3:
            assert g.k == 3 and g.first + 3 <= n3
            assert d3[g.first] == d3[g.first + 1] == d3[g.first + 2] == d3[g.first + 3] == chi
