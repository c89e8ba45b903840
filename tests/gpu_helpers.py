"""Shared helpers of the GPU parity tests (HIP path vs the CPU oracle)."""
import os

import numpy as np

import oracle
from paper_2403_02512_amd import qsv
from tests.parity_log import record

# Tolerances: state vectors by ||psi - psi_ref||_2 (||psi|| = 1); scalars
# relative to s = sum_t |c_t| of the observable (s bounds |<H>|, and with the
# per-slot factor below every derivative).
TOL = {qsv.C128: 1e-12, qsv.C64: 1e-5}


def dname(dt):
    return "c128" if dt == qsv.C128 else "c64"


def _case():
    # the running test's id (pytest sets it for the duration of each test)
    return os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]


def np_dtype(dt):
    return np.complex128 if dt == qsv.C128 else np.complex64


def gpu_run(ctx, n, ops, params, dtype=qsv.C128, psi0=None, options=None):
    """Apply ops on the GPU (from psi0, default |0..0>) and return the state."""
    for k, v in (options or {}).items():
        ctx.set_option(k, v)
    st = qsv.State(ctx, n, dtype)
    if psi0 is not None:
        st.from_numpy(psi0.astype(np_dtype(dtype)))
    qsv.apply(st, ops, params)
    out = st.to_numpy()
    st.close()
    return out


def reset_options(ctx):
    ctx.set_option(qsv.OPT_FUSION, 1)
    ctx.set_option(qsv.OPT_TILE_BITS, 0)
    ctx.set_option(qsv.OPT_TILE_BITS_ADJ, 0)
    ctx.set_option(qsv.OPT_LOW_BITS, 0)
    ctx.set_option(qsv.OPT_TILE_WS, 0)
    ctx.set_option(qsv.OPT_DENSE_MFMA, 0)
    ctx.set_option(qsv.OPT_LAYERS, 1)


def obs_scale(observables):
    return np.array([np.sum(np.abs(o.coeffs)) for o in observables])


def jac_bound(ops, n_params, observables):
    """|dJ[o, p]| bound: s_o * sum over slots of p of 2 |scale| (>= s_o)."""
    per_p = np.zeros(n_params)
    for o in ops:
        for p, sc in zip(o.param, o.scale):
            if p >= 0:
                per_p[p] += 2 * abs(sc)
    return np.outer(obs_scale(observables), np.maximum(per_p, 1.0))


def assert_state_close(got, ref, tol, what="", dtype=None):
    """||got - ref||_2 <= tol (states of norm 1); the error is recorded."""
    err = float(np.linalg.norm(got.astype(np.complex128) - ref))
    dt = dtype if dtype is not None else ("c64" if got.dtype == np.complex64 else "c128")
    record(_case(), "state " + what, dt if isinstance(dt, str) else dname(dt), err, tol)
    assert err <= tol, f"{what}: ||psi - psi_ref|| = {err:.3e} > {tol:.1e}"
    return err


def assert_rel_close(got, ref, scale, dt, what=""):
    """max |got - ref| / scale <= TOL[dt] (scale: the bounds of reading 10,
    sum |c_t| for expectation values, jac_bound for Jacobian entries); the
    achieved error is recorded."""
    err = float(np.max(np.abs(np.asarray(got) - np.asarray(ref)) / np.asarray(scale)))
    record(_case(), what, dname(dt), err, TOL[dt])
    assert err <= TOL[dt], f"{what}: relative error {err:.3e} > {TOL[dt]:.1e}"
    return err


def oracle_state(n, ops, params, psi0=None):
    return oracle.apply(n, ops, params, psi=psi0)
