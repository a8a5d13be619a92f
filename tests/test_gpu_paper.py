"""GPU runs of the paper's own Example 1 (Section 6): centred conservative
finite differences of (exp(-xy) u_x)_x + (exp(xy) u_y)_y on 148 x 148 interior
points, tol 1e-6, the residual checked at every step (d = 1), FP64 as in the
paper.  Compared with the oracle's run on the same seeded right-hand sides
(tests/golden/example1_oracle.json, written by make_example1_oracle.py) and
with the iteration counts of Table 1 (tests/golden/paper_example1.json)."""
import json
import os

import numpy as np
import pytest

from workloads import fd2d_variable, uniform_C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _b():
    from paper_1602_05033_amd import binding
    return binding


@pytest.mark.parametrize("s", [1, 4, 8])
def test_example1_against_oracle_and_table1(lib, s):
    b = _b()
    orc = json.load(open(os.path.join(GOLD, "example1_oracle.json")))["cases"][str(s)]
    paper = json.load(open(os.path.join(GOLD, "paper_example1.json")))
    op = fd2d_variable(148, lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y), "e1")
    C = uniform_C(op.n, s, 0)
    sol = b.lyap_solve(b.device_op(op), torch.from_numpy(np.ascontiguousarray(C)).cuda(), tol=1e-6,
                       storage=b.STORE_F64, check_every=1, two_pass=True)
    assert sol.status == b.OK
    # residual history: tight while the basis is still orthogonal (m <= 40;
    # at m = 80 the s = 4 runs already differ by 0.3%).
    # Over the window around m* both Lanczos runs have lost orthogonality and
    # agree only to the forward-instability level: the curve falls ~5% per
    # step there and the two runs differ by up to ~6% (about one step), so the
    # window is held to 15% and the first checked m with ||R||_F/||C||_F^2 <=
    # 1e-6 to two steps.
    gh = dict(zip(sol.hist_m, sol.hist_res))
    worst = 0.0
    for m, res in orc["hist"]:
        if m not in gh:          # past the GPU run's own stop (m* is compared below)
            continue
        dev = abs(gh[m] - res) / res
        assert dev <= (1e-6 if m <= 40 else 0.15), (m, gh[m], res)
        if m > 40:
            worst = max(worst, dev)
    print(f"s={s}: m {sol.m} (oracle {orc['m']}), largest late deviation {worst:.3f}")
    assert abs(sol.m - orc["m"]) <= 2, (sol.m, orc["m"])
    # Table 1's count with the paper's (unreproducible) random C
    ref = paper["iterations"][str(s)]
    assert abs(sol.m - ref) <= 0.03 * ref
    assert sol.hist_m == list(range(1, sol.m + 1))  # checked at every step
