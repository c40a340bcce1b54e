"""Admission policy of the solve server, replayed on the host (no GPU)."""
import numpy as np

from paper_1206_6409_amd import gencd as G


def _events(bytes_, arrival, service, start):
    ev = []
    for i, s in enumerate(start):
        if s >= 0:
            ev.append((s, 1, i))
            ev.append((s + service[i], -1, i))
    ev.sort(key=lambda e: (e[0], e[1]))  # releases before acquisitions at equal times
    return ev


def _check_invariants(arena, slots, bytes_, arrival, service, start):
    rb = [((b + 255) // 256) * 256 for b in bytes_]
    used, busy = 0, 0
    for t, kind, i in _events(bytes_, arrival, service, start):
        used += kind * rb[i]
        busy += kind
        assert used <= arena and busy <= slots
    for i, s in enumerate(start):
        if rb[i] > arena:
            assert s == -1
        else:
            assert s >= arrival[i]
    # FIFO: admitted requests start in arrival order
    ok = [i for i in range(len(start)) if start[i] >= 0]
    assert all(start[a] <= start[b] for a, b in zip(ok[:-1], ok[1:]))


def test_plan_unbounded_starts_on_arrival():
    rng = np.random.default_rng(0)
    n = 200
    arr = np.cumsum(rng.exponential(0.1, n))
    svc = rng.uniform(0.05, 0.5, n)
    b = rng.integers(1 << 10, 1 << 20, n)
    st = G.server_plan(1 << 40, 1000, b, arr, svc)
    np.testing.assert_allclose(st, arr)


def test_plan_single_slot_is_serial():
    arr = np.array([0.0, 0.1, 0.2, 5.0])
    svc = np.array([1.0, 1.0, 1.0, 1.0])
    st = G.server_plan(1 << 30, 1, [100, 100, 100, 100], arr, svc)
    np.testing.assert_allclose(st, [0.0, 1.0, 2.0, 5.0])


def test_plan_budget_backpressure_and_rejection():
    rng = np.random.default_rng(1)
    n = 300
    arr = np.cumsum(rng.exponential(0.05, n))
    svc = rng.uniform(0.1, 1.0, n)
    b = rng.integers(1 << 20, 64 << 20, n)
    b[17] = 2 << 30  # larger than the arena: rejected, must not block the rest
    arena = 256 << 20
    st = G.server_plan(arena, 6, b, arr, svc)
    assert st[17] == -1
    assert np.all(st[np.arange(n) != 17] >= 0)
    _check_invariants(arena, 6, b, arr, svc, st)
    # the budget binds: some requests had to wait
    assert np.any(st > arr + 1e-12)


def test_plan_head_of_line_blocks_smaller_followers():
    # the head needs the whole arena; the small one behind it waits for it
    arr = np.array([0.0, 0.0, 0.1])
    svc = np.array([1.0, 1.0, 0.1])
    b = np.array([600, 1000, 10]) * 256
    st = G.server_plan(1000 * 256, 4, b, arr, svc)
    np.testing.assert_allclose(st, [0.0, 1.0, 2.0])
