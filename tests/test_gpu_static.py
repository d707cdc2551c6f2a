"""GPU parity of the static (iSAX-style N(0,1)) encoding that the encoding phase contrasts
with its dynamic one (Section 3.1): the library's breakpoints against the oracle's
static_breakpoints, then codes, trees and queries stepwise against the oracle on the GPU's
breakpoints and codes, exactly as for the dynamic encoding."""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from parity import proj_bound
from test_gpu_parity import Case, check_codes, check_trees, run_and_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def static_case():
    w = wl.SMALL_MIXTURE
    return w, Case(w.data(), w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf,
                   encoding="static")


def test_static_breakpoints_within_bound(static_case):
    """B(z) = mu + sigma * Phi^-1((z-1)/Nr): the library's mean and standard deviation come
    from float32 projections, so each breakpoint may move by the projection error E of the
    sample (which bounds the change of both the mean and the population standard deviation)
    times (1 + |Phi^-1|), plus the float32 rounding of the result."""
    w, cs = static_case
    E_s = proj_bound(cs.X[cs.sid], cs.A).max(axis=0)
    E_all = proj_bound(cs.X, cs.A).max(axis=0)
    Bg, Bo = cs.B_gpu, cs.B_or
    from scipy.stats import norm
    z = norm.ppf(np.arange(1, w.Nr) / w.Nr)
    tol = E_s[:, None] * (1.0 + np.abs(z)[None, :]) + np.abs(Bo[:, 1:-1]) * 2.0 ** -23 + 1e-30
    assert np.all(np.abs(Bg[:, 1:-1] - Bo[:, 1:-1]) <= tol), float(
        (np.abs(Bg[:, 1:-1] - Bo[:, 1:-1]) / tol).max())
    assert np.all(np.abs(Bg[:, [0, -1]] - Bo[:, [0, -1]]) <= E_all[:, None] + 1e-30)
    # the mixture is not Gaussian: the static breakpoints are not its sample quantiles
    Bd = oracle.breakpoints(cs.H[cs.sid], w.Nr, cs.H.min(axis=0), cs.H.max(axis=0))
    assert np.abs(Bd[:, 1:-1] - Bo[:, 1:-1]).max() > 100 * tol.max()


def test_static_codes_and_trees(static_case):
    w, cs = static_case
    check_codes(cs)
    check_trees(cs)


@pytest.mark.parametrize("beta,r_min", [(0.1, 4.0), (0.02, 1.0)])
def test_static_query_stepwise(static_case, beta, r_min):
    w, cs = static_case
    run_and_compare(cs, cs.stepwise_oracle(), w.queries(), w.k, w.c, beta, r_min,
                    f"static b={beta}")
