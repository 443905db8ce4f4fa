"""Host logic of the shot queue, run without a GPU (SP_QUEUE_FAKE: the worker
thread admits, batches and retires shots but enqueues no device work).

Checks admission by budget and slots (resident bytes never exceed the
budget), FIFO order, rejection of shots that can never fit, isolation of a
failing shot and of a shot that computes a non-finite value (SP_ENUMERIC),
with full arena reclamation, and cancellation at shutdown.
"""

import ctypes

import pytest

from paper_2309_04671_amd import lib

FAKE_ARENA = 1 << 30                 # never dereferenced in fake mode


def desc(n, nsteps, dtype=lib.SP_F32):
    d = lib.sp_shot_desc()
    d.nx = d.ny = d.nz = n
    d.dtype = dtype
    d.nsteps = nsteps
    d.dt, d.dx = 1e-3, 10.0
    d.coeffs = lib.coeffs({"center": -1, "ax": [0.1] * 4, "ay": [0.1] * 4, "az": [0.1] * 4})
    d.v = 1 << 20
    d.nsrc = 1
    d.src_xyz[0][0] = d.src_xyz[0][1] = d.src_xyz[0][2] = n // 2
    d.src_amp = 1 << 21
    return d


def make_queue(arena_bytes, budget=0, slots=8, chunk=8):
    L = lib.load()
    cfg = lib.sp_queue_cfg(FAKE_ARENA, arena_bytes, budget, slots, chunk, lib.SP_QUEUE_FAKE, None)
    q = ctypes.c_void_p()
    lib.check(L.sp_queue_create(ctypes.byref(cfg), ctypes.byref(q)))
    return q


def submit(q, d):
    t = ctypes.c_uint64()
    rc = lib.load().sp_submit(q, ctypes.byref(d), ctypes.byref(t))
    return rc, t.value


def status(q, t):
    st = lib.sp_shot_status()
    rc = lib.load().sp_poll(q, t, ctypes.byref(st))
    return rc, st


def test_shot_bytes_counts_fields_velocity_and_records():
    L = lib.load()
    d32, d16 = desc(64, 10), desc(64, 10, lib.SP_F16)
    g32, g16 = lib.grid_init(64, 64, 64), lib.grid_init(64, 64, 64, lib.SP_F16)
    b32 = L.sp_shot_bytes(ctypes.byref(d32))
    b16 = L.sp_shot_bytes(ctypes.byref(d16))
    assert b32 >= 3 * g32.bytes and b16 >= 2 * g16.bytes + g32.bytes + L.sp_wave_meta_bytes(g16)
    assert b16 < b32
    bad = desc(64, 10)
    bad.nx = 0
    assert L.sp_shot_bytes(ctypes.byref(bad)) == -1


def test_budget_and_slots_bound_the_resident_set():
    L = lib.load()
    d = desc(48, 40)
    b = L.sp_shot_bytes(ctypes.byref(d))
    q = make_queue(1 << 30, budget=2 * b + b // 2, slots=3, chunk=7)    # two fit at once
    tickets = [submit(q, desc(48, 40 + 9 * k))[1] for k in range(7)]
    lib.check(L.sp_queue_drain(q))
    sts = [status(q, t)[1] for t in tickets]
    assert all(s.state == lib.SP_SHOT_DONE and s.error == 0 for s in sts)
    assert [s.steps_done for s in sts] == [40 + 9 * k for k in range(7)]
    # FIFO admission
    admits = [s.t_admit for s in sts]
    assert admits == sorted(admits)
    # at every admission instant at most two shots were resident
    for s in sts:
        live = [o for o in sts if o.t_admit <= s.t_admit < o.t_done]
        assert len(live) <= 2
    lib.check(L.sp_queue_destroy(q))


def test_slot_limit():
    L = lib.load()
    q = make_queue(1 << 30, slots=1, chunk=5)
    tickets = [submit(q, desc(32, 12))[1] for _ in range(4)]
    lib.check(L.sp_queue_drain(q))
    sts = [status(q, t)[1] for t in tickets]
    for a, b in zip(sts, sts[1:]):
        assert b.t_admit >= a.t_done           # one at a time
    lib.check(L.sp_queue_destroy(q))


def test_shot_that_can_never_fit_is_rejected():
    L = lib.load()
    q = make_queue(1 << 30, budget=1 << 20)
    rc, _ = submit(q, desc(64, 10))
    assert rc == lib.SP_EBUDGET and "budget" in lib.last_error()
    bad = desc(64, 0)
    assert submit(q, bad)[0] == lib.SP_EINVAL
    rc, _ = status(q, 12345)
    assert rc == lib.SP_EINVAL
    lib.check(L.sp_queue_destroy(q))


def test_failing_shot_is_isolated_and_memory_reclaimed(monkeypatch):
    L = lib.load()
    monkeypatch.setenv("SP_TEST_FAIL_TICKET", "2")
    d = desc(40, 30)
    b = L.sp_shot_bytes(ctypes.byref(d))
    q = make_queue(1 << 30, budget=3 * b, slots=4, chunk=4)
    tickets = [submit(q, desc(40, 30))[1] for _ in range(5)]
    lib.check(L.sp_queue_drain(q))
    sts = {t: status(q, t) for t in tickets}
    assert sts[2][0] == lib.SP_OK and sts[2][1].state == lib.SP_SHOT_FAILED
    assert sts[2][1].error == lib.SP_EDEVICE
    for t in tickets:
        if t != 2:
            assert sts[t][1].state == lib.SP_SHOT_DONE and sts[t][1].steps_done == 30
    # everything was returned: a shot needing the whole budget is admitted
    big = desc(40, 5)
    tickets2 = [submit(q, big)[1] for _ in range(3)]
    lib.check(L.sp_queue_drain(q))
    assert all(status(q, t)[1].state == lib.SP_SHOT_DONE for t in tickets2)
    lib.check(L.sp_queue_destroy(q))


def test_nonfinite_shot_fails_with_enumeric_and_memory_reclaimed(monkeypatch):
    # the fake executor reports a non-finite value for ticket 3 after its
    # first chunk: that shot ends FAILED / SP_ENUMERIC with the steps of
    # that chunk done, the others finish, and its memory returns
    L = lib.load()
    monkeypatch.setenv("SP_TEST_NONFINITE_TICKET", "3")
    d = desc(40, 30)
    b = L.sp_shot_bytes(ctypes.byref(d))
    q = make_queue(1 << 30, budget=3 * b, slots=4, chunk=4)
    tickets = [submit(q, desc(40, 30))[1] for _ in range(5)]
    lib.check(L.sp_queue_drain(q))
    sts = {t: status(q, t) for t in tickets}
    assert sts[3][0] == lib.SP_OK and sts[3][1].state == lib.SP_SHOT_FAILED
    assert sts[3][1].error == lib.SP_ENUMERIC and sts[3][1].steps_done == 4
    for t in tickets:
        if t != 3:
            assert sts[t][1].state == lib.SP_SHOT_DONE and sts[t][1].steps_done == 30
    big = desc(40, 5)
    tickets2 = [submit(q, big)[1] for _ in range(3)]
    lib.check(L.sp_queue_drain(q))
    assert all(status(q, t)[1].state == lib.SP_SHOT_DONE for t in tickets2)
    lib.check(L.sp_queue_destroy(q))


def test_destroy_finishes_running_and_cancels_queued():
    L = lib.load()
    q = make_queue(1 << 30, slots=1, chunk=1)
    tickets = [submit(q, desc(32, 400))[1] for _ in range(30)]
    lib.check(L.sp_queue_destroy(q))
    # the handle is gone; nothing to poll -- the call returning is the check
    assert len(tickets) == 30


def test_queue_config_validation():
    L = lib.load()
    q = ctypes.c_void_p()
    for cfg in (lib.sp_queue_cfg(None, 1 << 30, 0, 4, 4, lib.SP_QUEUE_FAKE, None),
                lib.sp_queue_cfg(FAKE_ARENA, 1 << 30, 0, 0, 4, lib.SP_QUEUE_FAKE, None),
                lib.sp_queue_cfg(FAKE_ARENA, 1 << 30, 0, 4, 0, lib.SP_QUEUE_FAKE, None),
                lib.sp_queue_cfg(FAKE_ARENA + 8, 1 << 30, 0, 4, 4, lib.SP_QUEUE_FAKE, None),
                lib.sp_queue_cfg(FAKE_ARENA, 1 << 20, 0, 4, 4, lib.SP_QUEUE_FAKE, None),
                lib.sp_queue_cfg(FAKE_ARENA, 1 << 30, 0, 4, 4, 64, None)):
        assert L.sp_queue_create(ctypes.byref(cfg), ctypes.byref(q)) == lib.SP_EINVAL


@pytest.mark.parametrize("dtype", [lib.SP_F32, lib.SP_F16, lib.SP_BF16])
def test_mixed_shapes_and_types(dtype):
    L = lib.load()
    q = make_queue(1 << 30, slots=16, chunk=6)
    shapes = [(128, 128, 128), (192, 192, 160), (64, 40, 30), (384, 96, 64)]
    tickets = []
    for k, (nx, ny, nz) in enumerate(shapes * 2):
        d = desc(8, 17 + k, dtype)
        d.nx, d.ny, d.nz = nx, ny, nz
        d.src_xyz[0][0], d.src_xyz[0][1], d.src_xyz[0][2] = nx // 2, ny // 2, nz // 2
        tickets.append(submit(q, d)[1])
    lib.check(L.sp_queue_drain(q))
    for k, t in enumerate(tickets):
        rc, st = status(q, t)
        assert rc == lib.SP_OK and st.state == lib.SP_SHOT_DONE and st.steps_done == 17 + k
    lib.check(L.sp_queue_destroy(q))


def test_library_log_reports_launch_choices_and_queue_events():
    # SP_LOG=1 (read once per process, hence a child process): the tile
    # choice of a launch and the queue's admissions, compositions and
    # retirements go to stderr
    import subprocess
    import sys
    import textwrap
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    code = textwrap.dedent('''
        import ctypes, sys
        sys.path.insert(0, %r)
        from tests.test_queue_host import desc, make_queue, submit
        from paper_2309_04671_amd import lib
        L = lib.load()
        q = make_queue(1 << 30, slots=2, chunk=5)
        for k in range(3):
            submit(q, desc(48, 12))
        lib.check(L.sp_queue_drain(q))
        lib.check(L.sp_queue_destroy(q))
        g = lib.grid_init(64, 64, 64)
        c = lib.coeffs({"center": -1, "ax": [0.1] * 4, "ay": [0.1] * 4, "az": [0.1] * 4})
        out = ctypes.c_int()
        L.sp_stencil_apply(ctypes.byref(g), ctypes.byref(c), 0, ctypes.c_void_p(1 << 30),
                           ctypes.c_void_p(1 << 40), ctypes.byref(out), None)
    ''' % root)
    env = dict(__import__("os").environ, SP_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[libstencil]")]
    assert sum("queue: admit ticket" in l for l in lines) == 3
    assert sum("queue: ticket" in l and " done " in l for l in lines) == 3
    assert any("queue: composition of " in l and "blocks per step" in l for l in lines)
    assert any("sp_stencil_apply: 64x64x64" in l and "z-chunk 1" in l for l in lines)
    # without SP_LOG nothing is printed
    env.pop("SP_LOG")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "[libstencil]" not in r.stderr
