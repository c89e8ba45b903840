"""The tuner: picks tile widths and the fusion form (layers, low bits) in
range, sets them on the context, and the circuit's results under the chosen
options still match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import jac_bound

pytestmark = pytest.mark.gpu


def test_autotune_qaoa_20q():
    ctx = qsv.Context(0)
    c = W.config3(n=20)
    st = qsv.State(ctx, 20)
    fb, ab = qsv.autotune(st, c.ops, c.params, c.observables)
    assert 10 <= fb <= 13 and 9 <= ab <= 12
    assert ctx.get_option(qsv.OPT_TILE_BITS) == fb and ctx.get_option(qsv.OPT_TILE_BITS_ADJ) == ab
    # the fusion form is chosen too: layers on/off, default or +-1 low bits
    assert ctx.get_option(qsv.OPT_LAYERS) in (0, 1) and ctx.get_option(qsv.OPT_LOW_BITS) in (0, 3, 5)
    # the state holds the circuit's output; gradients under the tuned options
    psi = oracle.apply(20, c.ops, c.params)
    assert np.linalg.norm(st.to_numpy() - psi) <= 1e-12
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    want = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)
    assert np.max(np.abs(jac - want) / jac_bound(c.ops, c.n_params, c.observables)[0]) <= 1e-12
    st.close()
    ctx.close()


def test_autotune_forward_only_and_errors():
    ctx = qsv.Context(0)
    c = W.random_circuit(12, 60, seed=3)
    st = qsv.State(ctx, 12, qsv.C64)
    fb, ab = qsv.autotune(st, c.ops, c.params)
    assert 10 <= fb <= 12 and ab == 0  # no observable: adjoint width untouched (default 0)
    assert ctx.get_option(qsv.OPT_LAYERS) in (0, 1) and ctx.get_option(qsv.OPT_LOW_BITS) in (0, 4, 6)
    with pytest.raises(qsv.QsvError):
        qsv.autotune(st, [W.op("RX", [13], (0, 1.0))], [0.1])
    assert ctx.get_option(qsv.OPT_TILE_BITS) == fb
    st.close()
    ctx.close()
