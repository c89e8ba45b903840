"""Error paths forced from the host (no kernel faults): an allocation limit
makes device allocations fail as out-of-memory, and an injected failure
stands in for a failed kernel launch.  A call that fails before its first
kernel leaves the state untouched, and the context stays usable."""
import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import assert_rel_close, jac_bound

pytestmark = pytest.mark.gpu

ERR_OOM, ERR_HIP = -4, -5


@pytest.fixture()
def ctx():
    c = qsv.Context(0)
    yield c
    c.close()


def test_state_allocation_over_limit_is_oom(ctx):
    ctx.set_option(qsv.OPT_TEST_ALLOC_LIMIT, 1 << 20)
    with pytest.raises(qsv.QsvError) as e:
        qsv.State(ctx, 17)                  # 2 MiB
    assert e.value.status == ERR_OOM
    st = qsv.State(ctx, 15)                 # 512 KiB: below the limit
    st.close()
    ctx.set_option(qsv.OPT_TEST_ALLOC_LIMIT, 0)
    qsv.State(ctx, 17).close()


@pytest.mark.parametrize("inplace", [False, True])
def test_adjoint_workspace_oom_leaves_state(ctx, inplace):
    n = 16
    c = W.random_circuit(n, 30, seed=3, n_params=4)
    obs = W.random_observables(n, np.random.default_rng(0), n_obs=1, n_terms=3)
    st = qsv.State(ctx, n)
    qsv.apply(st, c.ops, c.params)
    before = st.to_numpy()
    ctx.release_workspace()
    ctx.set_option(qsv.OPT_TEST_ALLOC_LIMIT, (1 << n) * 16 - 1)   # lambda / phi do not fit
    with pytest.raises(qsv.QsvError) as e:
        qsv.adjoint_jacobian(st, c.ops, c.params, obs, inplace=inplace)
    assert e.value.status == ERR_OOM
    np.testing.assert_array_equal(st.to_numpy(), before)
    ctx.set_option(qsv.OPT_TEST_ALLOC_LIMIT, 0)
    jac, _ = qsv.adjoint_jacobian(st, c.ops, c.params, obs, inplace=inplace)
    psi = oracle.apply(n, c.ops, c.params)
    assert_rel_close(jac, oracle.adjoint_jacobian(psi, c.ops, c.params, obs), jac_bound(c.ops, c.n_params, obs),
                     qsv.C128, "jacobian after recovery")
    st.close()


def test_injected_launch_failure(ctx):
    n = 14
    c = W.random_circuit(n, 40, seed=5, n_params=4)
    st = qsv.State(ctx, n)
    st.from_numpy(W.random_state(n, 1))
    before = st.to_numpy()
    # the first launch of the call fails: nothing ran, the state is as it was
    ctx.set_option(qsv.OPT_TEST_FAIL_LAUNCH, 1)
    with pytest.raises(qsv.QsvError) as e:
        qsv.apply(st, c.ops, c.params)
    assert e.value.status == ERR_HIP and "injected" in str(e.value)
    np.testing.assert_array_equal(st.to_numpy(), before)
    assert ctx.get_option(qsv.OPT_TEST_FAIL_LAUNCH) == 0      # spent
    # a failure in the middle of an adjoint sweep is reported (the state is
    # then undefined, as documented) and the next call works
    obs = W.random_observables(n, np.random.default_rng(1), n_obs=1, n_terms=2)
    ctx.set_option(qsv.OPT_TEST_FAIL_LAUNCH, 3)
    with pytest.raises(qsv.QsvError) as e:
        qsv.adjoint_jacobian(st, c.ops, c.params, obs)
    assert e.value.status == ERR_HIP
    st.reset(0)
    qsv.apply(st, c.ops, c.params)
    np.testing.assert_allclose(st.to_numpy(), oracle.apply(n, c.ops, c.params), atol=1e-12)
    st.close()


def test_bad_option_values(ctx):
    for opt in (qsv.OPT_TEST_ALLOC_LIMIT, qsv.OPT_TEST_FAIL_LAUNCH):
        with pytest.raises(qsv.QsvError):
            ctx.set_option(opt, -1)
