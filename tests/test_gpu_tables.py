"""Tables 1 and 2 of Sec. 4.1 on the GPU path (grids 32^2 ... 512^2, beyond
what the oracle steps in seconds).  The printed differences carry five
significant digits and the rates four decimals; the last printed digit also
carries the paper's own solver tolerance, so a row reproduces its entry when
the difference is within 2 units of the last printed digit and the rate within
1e-4.  Grids from 256^2 on run V(0,1) cycles (the App. B smoother alone is
unstable there and V(2,2) diverges).  Table 1's fourth row needs 102 400
first-order steps on 512^2 (about two minutes; the run prints its progress
every 20 000 steps); it is compared to four significant digits (the solve
there sits at the FP64 residual floor)."""
import json
import math
import os

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1208_2643_amd import convergence  # noqa: E402

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def unit(ref):
    """One unit in the 5th significant digit of a printed value."""
    return 10.0 ** (math.floor(math.log10(abs(ref))) - 4)


def check(rows, ref, nrows, digits5=None):
    """Rows 0 .. nrows-1; rows in `digits5` (default all) to the printed five
    digits (2 units) and rates to 1e-4, others to four digits and 1e-3."""
    assert len(rows) == nrows
    for k, row in enumerate(rows):
        d = ref["difference"][k]
        tight = digits5 is None or k in digits5
        tol_d = 2 * unit(d) if tight else 10 * unit(d)
        assert abs(row["difference"] - d) <= tol_d, (k, row["difference"], d)
        if ref["rate"][k] is not None:
            assert abs(row["rate"] - ref["rate"][k]) <= (1e-4 if tight else 1e-3), \
                (k, row["rate"], ref["rate"][k])


def test_table2_rows_1_4():
    """Second-order scheme, s = 0.05 h, grids 32^2 ... 512^2."""
    rows, runs = convergence.table(2, sizes=(32, 64, 128, 256, 512))
    assert all("error" not in r for r in runs)
    check(rows, GOLDEN["table2_scheme2"], 4)


@pytest.mark.timeout(600)
def test_table1_rows_1_4():
    """First-order scheme, s = 0.025 h^2, grids 32^2 ... 512^2, in the
    damped-wave form that reproduces the printed values (beta = M = 1/0.9 in
    the stepped form).  Rows 1-3 to five digits; the fourth (102 400 steps on
    512^2) to four."""
    rows, runs = convergence.table(1, sizes=(32, 64, 128, 256, 512))
    assert all("error" not in r for r in runs)
    check(rows, GOLDEN["table1_scheme1"], 4, digits5=(0, 1, 2))
