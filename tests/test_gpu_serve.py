"""GPU tests of the continuous-batching shot queue.

Bars:
 * every shot's traces and final field are bit-identical alone in the queue,
   in a mix of shapes and storage types, with graph replay or eager launches,
   and against a direct sp_wave_step run (same kernels, same arithmetic);
 * a queued FP32 shot matches the FP64 oracle (multi-step rel-L2 <= 1e-4);
 * the four served shapes up to 384x384x256, FP32 and FP16 in one mix,
   equal direct runs bit for bit;
 * requests submitted while others run are admitted before those finish;
 * a shot that blows up (an infinite source amplitude) ends FAILED with
   SP_ENUMERIC, FP32 or FP16, while its neighbours in the batch finish with
   the results they have alone.
"""

import time

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import errors

pytestmark = pytest.mark.gpu


def _shots(serve, lib, specs):
    out = []
    for k, (nx, ny, nz, dtype, nsteps) in enumerate(specs):
        p = synth.wave_problem(nx, ny, nz, nsteps, seed=100 + k,
                               src=synth.random_points(nx, ny, nz, 1, 200 + k, margin=4))
        rec = synth.receiver_plane(nx, ny, min(8, nz - 1), 4)
        out.append((p, serve.Shot(p["v"], p["dt"], p["dx"], nsteps, synth.star25_coeffs(), p["src"],
                                  p["amp"] * 1e3, rec=rec, dtype=dtype)))
    return out


SPECS = [(64, 48, 40, 0, 37), (100, 60, 50, 1, 45), (72, 72, 36, 2, 29), (130, 33, 70, 0, 52),
         (96, 80, 48, 1, 33)]


def _run(serve, lib, specs, slots, flags=0, chunk=8):
    cl = serve.ServeClient(arena_bytes=2 << 30, max_slots=slots, chunk_steps=chunk, flags=flags)
    shots = _shots(serve, lib, specs)
    for _, s in shots:
        cl.submit(s)
    cl.drain()
    for _, s in shots:
        done, st = cl.poll(s.ticket)
        assert done and st.state == lib.SP_SHOT_DONE, (st.state, st.error)
    res = [(s.traces.cpu().numpy(), s.final.cpu().numpy()) for _, s in shots]
    cl.close()
    return shots, res


def test_solo_mix_graph_eager_and_direct_are_identical(gpu_lib):
    from paper_2309_04671_amd import fields, lib, serve
    _, mix = _run(serve, lib, SPECS, slots=8)
    _, solo = _run(serve, lib, SPECS, slots=1)
    _, eager = _run(serve, lib, SPECS, slots=8, flags=lib.SP_QUEUE_EAGER, chunk=5)
    for k in range(len(SPECS)):
        for a, b, c in zip(mix[k], solo[k], eager[k]):
            assert np.array_equal(a, b) and np.array_equal(a, c), k
    # direct single-grid runs of the same shots
    shots = _shots(serve, lib, SPECS)
    for k, (p, s) in enumerate(shots):
        nx, ny, nz, dtype, nsteps = SPECS[k]
        g = lib.grid_init(nx, ny, nz, dtype)
        gv = lib.grid_init(nx, ny, nz)
        V = fields.Field(gv).set_interior(p["v"])
        ws = fields.WaveState(g)
        tr = torch.zeros_like(s.traces)
        lib.sp_wave_step(g, lib.coeffs(synth.star25_coeffs()), p["dt"], p["dx"], gv, V.ptr, ws.st,
                         nsteps, src=lib.make_sources(p["src"], s.amp.data_ptr(), 1),
                         rec=lib.make_receivers(len(s.rec), s.rec_d.data_ptr(), tr.data_ptr(),
                                                len(s.rec)))
        torch.cuda.synchronize()
        assert np.array_equal(tr.cpu().numpy(), mix[k][0]), k
        assert np.array_equal(ws.decoded().astype(np.float32), mix[k][1]), k


def test_queued_fp32_shot_matches_oracle(gpu_lib):
    from paper_2309_04671_amd import lib, serve
    spec = [(80, 56, 44, 0, 60)]
    shots, res = _run(serve, lib, spec, slots=4)
    p, s = shots[0]
    co = synth.star25_coeffs()
    ref = oracle.wave_run(co, p["v"], p["dt"], p["dx"], 60, src=p["src"],
                          amp=s.amp.cpu().double().numpy(), rec=s.rec)
    e = errors(res[0][1], oracle.interior(ref["cur"]))
    et = errors(res[0][0], ref["traces"])
    print("queued shot vs oracle:", e, et)
    assert e["rel_l2"] <= 1e-4 and et["rel_l2"] <= 1e-4


def test_late_requests_join_running_batch(gpu_lib):
    from paper_2309_04671_amd import lib, serve
    cl = serve.ServeClient(arena_bytes=2 << 30, max_slots=8, chunk_steps=8)
    first = _shots(serve, lib, [(384, 384, 256, 0, 2000)])[0][1]      # ~0.2 s of work
    # the late requests are built beforehand, so that nothing but the
    # sleep separates their submission from the first one's
    late = [s for _, s in _shots(serve, lib, [(96, 96, 64, 1, 40), (64, 64, 64, 0, 30)])]
    cl.submit(first)
    time.sleep(0.02)
    for s in late:
        cl.submit(s)
    cl.drain()
    _, st0 = cl.poll(first.ticket)
    for s in late:
        done, st = cl.poll(s.ticket)
        assert done and st.state == lib.SP_SHOT_DONE
        print("late shot admitted %.3f s after the first, first done %.3f s later" %
              (st.t_admit - st0.t_admit, st0.t_done - st.t_admit))
        assert st.t_admit < st0.t_done          # admitted while the first still ran
        assert st.t_done < st0.t_done           # and finished before it
    cl.close()


def test_c4_shapes_mixed_equal_direct_runs(gpu_lib):
    # The four served grid shapes, FP32 and FP16 alternating, in one mix:
    # every result equals a direct sp_wave_step run bit for bit, and the
    # 128^3 FP32 shot matches the FP64 oracle.
    from paper_2309_04671_amd import fields, lib, serve
    specs = [(128, 128, 128, 0, 220), (192, 192, 160, 1, 240), (256, 256, 256, 0, 200),
             (384, 384, 256, 1, 210)]
    shots, res = _run(serve, lib, specs, slots=8, chunk=16)
    for k, (p, s) in enumerate(shots):
        nx, ny, nz, dtype, nsteps = specs[k]
        g = lib.grid_init(nx, ny, nz, dtype)
        gv = lib.grid_init(nx, ny, nz)
        V = fields.Field(gv).set_interior(p["v"])
        ws = fields.WaveState(g)
        tr = torch.zeros_like(s.traces)
        lib.sp_wave_step(g, lib.coeffs(synth.star25_coeffs()), p["dt"], p["dx"], gv, V.ptr, ws.st,
                         nsteps, src=lib.make_sources(p["src"], s.amp.data_ptr(), 1),
                         rec=lib.make_receivers(len(s.rec), s.rec_d.data_ptr(), tr.data_ptr(),
                                                len(s.rec)))
        torch.cuda.synchronize()
        assert np.array_equal(tr.cpu().numpy(), res[k][0]), k
        assert np.array_equal(ws.decoded().astype(np.float32), res[k][1]), k
        del ws, V
    p, s = shots[0]
    ref = oracle.wave_run(synth.star25_coeffs(), p["v"], p["dt"], p["dx"], 220, src=p["src"],
                          amp=s.amp.cpu().double().numpy(), rec=s.rec)
    e = errors(res[0][1], oracle.interior(ref["cur"]))
    print("served 128^3 FP32 shot vs oracle:", e)
    assert e["rel_l2"] <= 1e-4


@pytest.mark.parametrize("bad_dtype", [0, 1])
def test_blown_up_shot_fails_with_enumeric_neighbours_unaffected(gpu_lib, bad_dtype):
    from paper_2309_04671_amd import lib, serve
    specs = [(64, 48, 40, 0, 37), (100, 60, 50, 1, 45), (72, 72, 36, bad_dtype, 29)]
    _, solo = _run(serve, lib, specs[:2], slots=1)
    cl = serve.ServeClient(arena_bytes=2 << 30, max_slots=8, chunk_steps=8)
    shots = _shots(serve, lib, specs)
    bad = shots[2][1]
    bad.amp[3:] = float("inf")                 # u^4 is infinite at the source
    for _, s in shots:
        cl.submit(s)
    cl.drain()
    done, st = cl.poll(bad.ticket)
    assert done and st.state == lib.SP_SHOT_FAILED and st.error == lib.SP_ENUMERIC, (st.state, st.error)
    assert st.steps_done == 8                  # found at the end of the first chunk
    for k in range(2):
        done, st = cl.poll(shots[k][1].ticket)
        assert done and st.state == lib.SP_SHOT_DONE
        assert np.array_equal(shots[k][1].traces.cpu().numpy(), solo[k][0]), k
        assert np.array_equal(shots[k][1].final.cpu().numpy(), solo[k][1]), k
    cl.close()
