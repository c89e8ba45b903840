"""qsv_expval_noalloc (no device allocation: static per-device scratch)
through the C ABI, against qsv_expval on the same states: two calls in a
row, the second smaller, in both precisions; the library's own device
buffers stay empty; observables beyond the scratch are rejected before any
device work."""
import numpy as np
import pytest

from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import TOL, assert_rel_close, obs_scale

pytestmark = pytest.mark.gpu

ERR_ARG = -1


def _grouped(n, sizes, seed):
    """x-groups of the given sizes (the first diagonal): many-term groups take
    the byte-table path, small ones the term loop."""
    rng = np.random.default_rng(seed)
    words, coeffs = [], []
    for gi, size in enumerate(sizes):
        x = 0 if gi == 0 else int(rng.integers(1, 1 << n))
        zs = set()
        while len(zs) < size:
            z = int(rng.integers(0, 1 << n))
            if x or z:
                zs.add(z)
        for z in sorted(zs):
            w = []
            for q in range(n):
                b = n - 1 - q
                xb, zb = (x >> b) & 1, (z >> b) & 1
                w.append("Y" if xb and zb else "X" if xb else "Z" if zb else "I")
            words.append("".join(w))
            coeffs.append(float(rng.normal()))
    return W.PauliSum(np.array(coeffs), words)


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
def test_noalloc_matches_expval_two_calls(dt):
    ctx = qsv.Context(0)
    try:
        for n, obs in ((20, [_grouped(20, (40, 17, 3, 1), 1), _grouped(20, (5, 5), 2),
                             W.random_pauli_sum(20, 60, np.random.default_rng(3))]),
                       (12, [W.random_pauli_sum(12, 3, np.random.default_rng(4))])):
            st = qsv.State(ctx, n, dt)
            c = W.random_circuit(n, 40, seed=n, n_params=4)
            qsv.apply(st, c.ops, c.params)
            ws = ctx.workspace_bytes()
            got = qsv.expval_noalloc(st, obs)
            # the allocation-free call grew none of the library's device buffers
            assert ctx.workspace_bytes() == ws
            want = qsv.expval(st, obs)
            assert_rel_close(got, want, obs_scale(obs), dt, f"noalloc vs expval n={n}")
            st.close()
    finally:
        ctx.close()


def test_noalloc_rejects_observables_beyond_scratch():
    ctx = qsv.Context(0)
    try:
        n = 20
        st = qsv.State(ctx, n)
        rng = np.random.default_rng(9)
        # ~170 000 single-term x-groups: tables of about 11 MB > 8 MiB of scratch
        m = 170_000
        xs = rng.integers(1, 1 << n, m, dtype=np.int64)
        zs = rng.integers(0, 1 << n, m, dtype=np.int64)
        letters = np.array(["I", "X", "Z", "Y"])
        bits = [((xs >> (n - 1 - q)) & 1) + 2 * ((zs >> (n - 1 - q)) & 1) for q in range(n)]
        words = ["".join(t) for t in zip(*[letters[b] for b in bits])]
        big = W.PauliSum(rng.normal(size=m), words)
        with pytest.raises(qsv.QsvError) as e:
            qsv.expval_noalloc(st, [big])
        assert e.value.status == ERR_ARG and "scratch" in str(e.value)
        # a following call of normal size works
        small = [W.random_pauli_sum(n, 4, rng)]
        assert_rel_close(qsv.expval_noalloc(st, small), qsv.expval(st, small), obs_scale(small), qsv.C128,
                         "noalloc after a rejected call")
        st.close()
    finally:
        ctx.close()
