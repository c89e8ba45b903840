"""Shot sampling (qsv_sample) against the oracle's inverse transform on the
same state and the same uniforms.  Indices must agree except where u lands
within rounding of a boundary of the running sum (the two sides sum in
different orders); every returned index must have non-zero probability."""
import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = qsv.Context(0)
    yield c
    c.close()


def _check(psi, u, got):
    """psi: the state the device sampled (complex128 copy)."""
    p = np.abs(psi) ** 2
    want = oracle.sample(psi, u)
    cdf = np.cumsum(p)
    tot = cdf[-1]
    assert np.all(p[got] > 0)
    bad = np.nonzero(got != want)[0]
    for k in bad:  # allowed only at a boundary within rounding
        t = u[k] * tot
        lo = cdf[got[k] - 1] if got[k] > 0 else 0.0
        assert lo - 1e-12 * tot <= t <= cdf[got[k]] + 1e-12 * tot, (k, got[k], want[k])
    return len(bad)


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
@pytest.mark.parametrize("n", [1, 3, 6, 7, 11, 14])
def test_sample_random_states(ctx, n, dt):
    c = W.random_circuit(n, 40, seed=100 + n)
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, c.ops, c.params)
    psi = st.to_numpy().astype(np.complex128)
    u = np.random.default_rng(n).random(3000)
    u[:3] = [0.0, 0.5, np.nextafter(1.0, 0.0)]
    got = qsv.sample(st, u)
    assert _check(psi, u, got) <= 3
    st.close()


def test_sample_basis_ghz_and_errors(ctx):
    st = qsv.State(ctx, 9)
    st.reset(300)
    assert np.all(qsv.sample(st, [0.0, 0.3, 0.99]) == 300)
    st.reset(0)
    g = W.ghz(9)
    qsv.apply(st, g.ops, g.params)
    got = qsv.sample(st, [0.1, 0.4, 0.6, 0.9])
    assert list(got[[0, 1]]) == [0, 0] and list(got[[2, 3]]) == [511, 511]
    with pytest.raises(qsv.QsvError):
        qsv.sample(st, [1.0])
    with pytest.raises(qsv.QsvError):
        qsv.sample(st, [-0.1])
    assert qsv.sample(st, []).size == 0
    st.close()


def test_sample_frequencies(ctx):
    c = W.random_circuit(5, 50, seed=7)
    st = qsv.State(ctx, 5)
    qsv.apply(st, c.ops, c.params)
    p = np.abs(st.to_numpy()) ** 2
    u = np.random.default_rng(1).random(200000)
    f = np.bincount(qsv.sample(st, u), minlength=32) / u.size
    assert np.all(np.abs(f - p) <= 5 * np.sqrt(p * (1 - p) / u.size) + 1e-12)
    st.close()


def test_sample_28q_qaoa_state(ctx):
    """The benchmark's 28-qubit state (large chunks, 2^12 amplitudes each)."""
    c = W.config3()
    st = qsv.State(ctx, 28)
    qsv.apply(st, c.ops, c.params)
    u = np.random.default_rng(5).random(4096)
    got = qsv.sample(st, u)
    psi = st.to_numpy()
    assert _check(psi, u, got) <= 3
    st.close()
    ctx.release_workspace()
