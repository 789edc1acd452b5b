"""The small exponential of the Lanczos approximation (Eq. zk) on the GPU:
y = exp(-i tau T) e_1 for a tridiagonal T, evaluated by the Chebyshev series
the Lanczos stop test uses, against the oracle's eigendecomposition of T.

Cases span orders k from 1 to the 1024 cap and |tau| r (r the Gershgorin
half-width of T, the series length) from 50 to 6e4: the all-electron-like
workload's smallest cells reach a few 1e4 at its dt, beyond the 6,144-term
table the series had before.  y has unit 2-norm (exp(-i tau T) is unitary),
so the bar is absolute: 1e-10.  Beyond the table the call reports EINVAL.
"""
import numpy as np
import pytest

from oracle.lanczos import tridiag_expm_e1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tridiag(k, tau, tau_r, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, k)
    b = rng.uniform(0.05, 1.0, max(k - 1, 0))
    rad = np.zeros(k)
    if k > 1:
        rad[:-1] += b
        rad[1:] += b
    r = 0.5 * ((a + rad).max() - (a - rad).min())
    s = tau_r / (abs(tau) * r) if r > 0 else tau_r / abs(tau)
    return a * s, b * s


@pytest.mark.parametrize("k,tau,tau_r", [(1, 0.3, 5.0), (8, 0.05, 50.0), (40, 0.005, 3.0e3), (60, 0.005, 2.0e4),
                                         (64, -0.005, 2.0e4), (65, 0.005, 1.2e4), (200, 0.005, 1.2e4),
                                         (700, -0.05, 4.0e4), (1024, 0.005, 6.0e4)])
def test_small_exponential_matches_oracle(k, tau, tau_r):
    from paper_1810_13130_amd import tdfe
    a, b = _tridiag(k, tau, tau_r, 1000 + k)
    print(f"[small-exp] k={k} tau={tau} |tau| r={tau_r:g}", flush=True)
    y, terms = tdfe.tridiag_expm(a, b, tau)
    ref = tridiag_expm_e1(a, b, tau)
    assert terms >= (tau_r if k > 1 else 0)
    assert abs(np.linalg.norm(y) - 1.0) <= 1e-10
    assert np.abs(y - ref).max() <= 1e-10


def test_small_exponential_beyond_the_table_is_reported():
    from paper_1810_13130_amd import tdfe
    a, b = _tridiag(100, 0.005, 1.0e5, 7)
    with pytest.raises(tdfe.TdfeError) as e:
        tdfe.tridiag_expm(a, b, 0.005)
    assert e.value.status == tdfe.EINVAL
