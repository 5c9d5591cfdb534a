"""The oracle's loops may run on several host threads; its results must not
depend on how many.  Also: the checkpointed reverse sweep gives exactly the
results of the one that keeps every state.  Both run on the CPU."""
import numpy as np

import oracle
from paper_2006_01748_amd import workloads as wl


def test_threads_do_not_change_bits():
    g = np.random.Generator(np.random.PCG64(wl.BASE_SEED + 71))
    nx, ny = 203, 131
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = wl.PARAMS_REF
    dt = oracle.stable_dt(a, b, c, prm[2], 0.9)
    prev = oracle.set_threads()
    try:
        oracle.set_threads(1)
        one = oracle.run(u, v, w, a, b, c, prm, dt, 25, mass_every=5)
        oracle.set_threads(max(4, prev))
        many = oracle.run(u, v, w, a, b, c, prm, dt, 25, mass_every=5)
    finally:
        oracle.set_threads(prev)
    assert all(np.array_equal(x, y) for x, y in zip(one, many))


def test_checkpointed_sweep_equals_full_sweep():
    g = np.random.Generator(np.random.PCG64(wl.BASE_SEED + 72))
    nx, ny, steps = 37, 23, 25
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = wl.PARAMS_REF
    dt = oracle.stable_dt(a, b, c, prm[2], 0.9)
    lam = [g.standard_normal((ny, nx)) for _ in range(3)]
    full = oracle.adjoint_run(u, v, w, a, b, c, prm, dt, steps, lam)
    for every in (1, 6, 25, 40):   # ragged last segment, one segment, longer than the run
        ck = oracle.adjoint_run_ckpt(u, v, w, a, b, c, prm, dt, steps, lam, every)
        for x, y in zip(full[:2], ck[:2]):
            assert all(np.array_equal(p, q) for p, q in zip(x, y)), every
        assert np.array_equal(full[2], ck[2]), every
