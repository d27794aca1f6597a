"""The library's exponential-variogram fit (host arithmetic behind the C ABI,
no GPU needed) against the oracle's fit on the same points: both minimise the
same weighted residual, by different searches."""
import numpy as np
import pytest

import paper_2505_22675_amd as ag


@pytest.mark.parametrize("a_true,c_true,noise", [(13.7, 7.3, 0.0), (40.0, 900.0, 0.03),
                                                 (3.0, 0.5, 0.1), (250.0, 12.0, 0.02)])
def test_fit_matches_oracle(orc, a_true, c_true, noise):
    rng = np.random.default_rng(int(a_true * 10))
    h = np.concatenate([np.arange(1, 33) * 2.0, np.arange(1, 33) * 2.5])
    g = c_true * (1.0 - np.exp(-h / a_true)) * (1.0 + noise * rng.standard_normal(h.size))
    w = rng.integers(1000, 100000, h.size).astype(np.float64)
    a, c, rc = ag.auv_fit_exponential(h, g, w)
    oa, oc, orc_rc = orc.fit_exponential(h, g, w)
    assert rc == ag.AUV_OK and orc_rc == 0
    assert a == pytest.approx(oa, rel=1e-6)
    assert c == pytest.approx(oc, rel=1e-6)
    if noise == 0.0:
        assert a == pytest.approx(a_true, rel=1e-7)


def test_fit_edge_cases():
    h = np.arange(1, 21) * 1.0
    _, _, rc = ag.auv_fit_exponential(h, 0.3 * h, np.ones_like(h))   # linear: no sill
    assert rc == ag.AUV_ERR_RANGE
    with pytest.raises(ag.AuvError):
        ag.auv_fit_exponential(h[:1], h[:1], np.ones(1))              # one point
    g = 4.0 * (1.0 - np.exp(-h / 9.0))
    w = np.ones_like(h)
    g[2], w[5] = np.nan, 0.0
    a, c, rc = ag.auv_fit_exponential(h, g, w)
    assert rc == ag.AUV_OK and a == pytest.approx(9.0, rel=1e-7) and c == pytest.approx(4.0, rel=1e-7)
