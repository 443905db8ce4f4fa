"""The C ABI used from plain C: the header compiles as strict C99, a C client
links against the library and gets its documented layout and refusals on the
CPU, and on the GPU the client's own fields, allocated and filled in C, give
the oracle's sweep and leapfrog."""

import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests.c_client import ROOT, client_binary, compile_client, run_client


def _coeff_file(path, co):
    w = [co["center"]] + list(co["ax"]) + list(co["ay"]) + list(co["az"])
    np.asarray(w, np.float64).tofile(path)


def test_header_is_strict_c99():
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                    "-x", "c", os.path.join(ROOT, "include", "stencil.h")], check=True)


def test_c_client_host_checks(tmp_path):
    exe = compile_client(str(tmp_path / "abi_client"))
    r = run_client("host", binary=exe)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "host ok"
    r = run_client("apply", binary=exe)
    assert r.returncode == 1 and "expected" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(23, 37, 70), (64, 64, 64)])
def test_c_client_apply_matches_oracle(gpu_lib, tmp_path, shape):
    nz, ny, nx = shape
    # integer weights and fields: every partial sum is exact in FP32
    u = synth.integer_field(shape, 3, bound=170)
    co = synth.integer_coeffs()
    u.astype(np.float32).tofile(tmp_path / "u.f32")
    _coeff_file(tmp_path / "c.f64", co)
    exe = client_binary(str(tmp_path))
    r = run_client("apply", nx, ny, nz, 1, tmp_path / "u.f32", tmp_path / "c.f64", tmp_path / "out.f32",
                   binary=exe)
    assert r.returncode == 0, r.stderr
    assert "result in v" in r.stdout
    got = np.fromfile(tmp_path / "out.f32", np.float32).reshape(shape)
    assert np.array_equal(got.astype(np.float64), oracle.laplacian(oracle.padded(u), co))
    # two sweeps with the eighth-order weights: the result is back in u
    u = synth.uniform_field(shape, 4)
    co = synth.star25_coeffs()
    u.tofile(tmp_path / "u.f32")
    _coeff_file(tmp_path / "c.f64", co)
    r = run_client("apply", nx, ny, nz, 2, tmp_path / "u.f32", tmp_path / "c.f64", tmp_path / "out.f32",
                   binary=exe)
    assert r.returncode == 0, r.stderr
    assert "result in u" in r.stdout
    got = np.fromfile(tmp_path / "out.f32", np.float32).reshape(shape)
    ru, rv, in_v = oracle.stencil_apply(oracle.padded(u), oracle.padded(np.zeros(shape)), co, 2)
    assert in_v == 0
    ref = oracle.interior(ru)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 2e-5


@pytest.mark.gpu
def test_c_client_wave_matches_oracle(gpu_lib, tmp_path):
    nx, ny, nz, nsteps = 61, 45, 38, 40
    v = synth.layered_velocity(nx, ny, nz, 2)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    w = synth.ricker(nsteps, dt, 15.0).astype(np.float32)
    sx, sy, sz = 30, 22, 19
    v.astype(np.float32).tofile(tmp_path / "v.f32")
    _coeff_file(tmp_path / "c.f64", co)
    w.tofile(tmp_path / "amp.f32")
    r = run_client("wave", nx, ny, nz, nsteps, repr(dt), repr(dx), tmp_path / "v.f32", tmp_path / "c.f64",
                   sx, sy, sz, tmp_path / "amp.f32", tmp_path / "out.f32", binary=client_binary(str(tmp_path)))
    assert r.returncode == 0, r.stderr
    got = np.fromfile(tmp_path / "out.f32", np.float32).reshape(nz, ny, nx)
    res = oracle.wave_run(co, v, dt, dx, nsteps, src=np.array([[sx, sy, sz]], np.int32),
                          amp=w.astype(np.float64)[:, None])
    ref = oracle.interior(res["cur"])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4
