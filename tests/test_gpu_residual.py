"""Parity of the HIP residual E(u) (through the C ABI) against the FP64 oracle.

Gate (FP64): |E_gpu - E_oracle| <= 1e-11 * scale per entry, where scale is the
sum of the absolute values of the terms that make up that entry (floored at 1).
"""
import numpy as np
import pytest
import torch

from oracle import residual as oresidual
from oracle.equations import residual_rows, row_scale, zeta_grid
from oracle.solve import jvp_complex, jvp_fd
from paper_1403_5044_amd import api, inputs

from gpu_common import dev, gprob, gpu_residual, host, log, oprob

pytestmark = pytest.mark.gpu

TOL64 = 1e-11

SMALL_CASES = [
    # (name, problem settings)
    ("tiny9x5", dict(N=9, M=5, x1=-3.0, xN=3.0, yM=2.0, F=0.7, eps=0.3)),
    ("31x11", inputs.W31X11),
    ("even40x9", dict(N=40, M=9, x1=-6.0, xN=5.0, yM=4.0, F=0.9, eps=0.2)),
    ("simpson13x7", dict(N=13, M=7, x1=-4.0, xN=4.0, yM=3.0, F=0.7, eps=0.4,
                         weights="simpson")),
    ("notaknot61x21", dict(N=61, M=21, x1=-16.0, xN=8.0, yM=12.0, F=0.6, eps=0.2,
                           spline_bc="notaknot")),
    ("ragged97x13", dict(N=97, M=13, x1=-10.0, xN=14.0, yM=6.0, F=1.0, eps=0.1)),
]


def _check(name, p, u, E, tol=TOL64):
    op = oprob(p)
    Eo = oresidual(op, u)
    sc = row_scale(op, u)
    err = np.abs(E - Eo) / sc
    log(f"{name}: max rel err {err.max():.3e} (entries {E.size})")
    assert np.all(np.isfinite(E))
    assert err.max() <= tol, (name, int(err.argmax()), err.max())
    return err.max()


@pytest.mark.parametrize("name,cfg", [("31x11", inputs.W31X11), ("181x61", inputs.W181X61)])
def test_flat_state_without_source_is_exactly_zero(name, cfg):
    p = gprob(cfg, eps=0.0)
    E = gpu_residual(p, inputs.flat_state(p.N, p.M))
    log(f"{name}: max |E| = {np.abs(E).max()}")
    assert np.all(E == 0.0)


@pytest.mark.parametrize("name,cfg", SMALL_CASES)
def test_residual_parity_small_meshes(name, cfg):
    p = gprob(cfg)
    for seed, u in enumerate([inputs.flat_state(p.N, p.M),
                              inputs.perturbed(inputs.flat_state(p.N, p.M), 1e-3, 1),
                              inputs.smooth_state(p.N, p.M, 0.05, 2),
                              inputs.smooth_state(p.N, p.M, 0.2, 3)]):
        E = gpu_residual(p, u)
        _check(f"{name}/state{seed}", p, u, E)


def test_residual_parity_181x61_batch_sampled():
    """181 x 61, 16 states = linear solution + N(0, 1e-3^2): E1/E4/E6
    compared everywhere, E2 at 48 sampled collocation points per state (plus the
    corners of the collocation grid)."""
    p = gprob(inputs.W181X61)
    op = oprob(p)
    NM = p.N * p.M
    rng = np.random.default_rng(123)
    corners = [NM + 1, NM + p.N - 1, NM + (p.M - 1) * p.N + 1, 2 * NM - 1]
    worst = 0.0
    for s, u in enumerate(inputs.batch_181x61(16)):
        E = gpu_residual(p, u)
        assert np.all(np.isfinite(E))
        e2 = NM + rng.integers(0, p.M, 48) * p.N + rng.integers(1, p.N, 48)
        rows = np.unique(np.concatenate([np.arange(NM), np.arange(NM, 2 * NM, p.N),
                                         e2, corners]))
        Eo, sc = residual_rows(op, u, rows)
        err = (np.abs(E[rows] - Eo) / sc).max()
        worst = max(worst, err)
        assert err <= TOL64, (s, err)
    log(f"181x61 batch: worst rel err {worst:.3e}")


def test_residual_is_deterministic():
    p = gprob(inputs.W181X61)
    u = dev(inputs.batch_181x61(1)[0])
    a = host(api.residual(p, u))
    b = host(api.residual(p, u))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name,cfg", [("31x11", inputs.W31X11),
                                      ("ragged97x13", SMALL_CASES[5][1])])
def test_fp32_kahan_residual_error_is_small(name, cfg):
    p = gprob(cfg)
    u = inputs.smooth_state(p.N, p.M, 0.05, 5)
    E32 = gpu_residual(p.with_(precision="fp32"), u)
    op = oprob(p)
    Eo = oresidual(op, u)
    err = (np.abs(E32 - Eo) / row_scale(op, u)).max()
    log(f"{name}: FP32-Kahan max rel err vs FP64 oracle {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("N", [1025, 2050])
def test_residual_parity_beyond_one_lds_segment(N):
    """Meshes wider than the 1024 source records that one LDS stage holds: the pair
    kernels take a row in segments (1025 = 1024 + 1, 2050 = 1024 + 1024 + 2).  FP64
    against the oracle at the usual gate, FP32-Kahan within 2^-19 of the row scale
    (the bound of the FP32 reading), and the batched residual bitwise equal to the
    single one."""
    cfg = dict(N=N, M=5, x1=-20.0, xN=20.0, yM=2.0, F=0.7, eps=0.2)
    p = gprob(cfg)
    u = inputs.smooth_state(p.N, p.M, 0.05, 6)
    E = gpu_residual(p, u)
    _check(f"wide{N}x5", p, u, E)
    op = oprob(p)
    E32 = gpu_residual(p.with_(precision="fp32"), u)
    err32 = (np.abs(E32 - oresidual(op, u)) / row_scale(op, u)).max()
    log(f"wide{N}x5: FP32-Kahan max rel err vs FP64 oracle {err32:.3e}")
    assert err32 <= 2.0 ** -19
    probs = [p, api.Problem(31, 11, -8.0, 8.0, 8.0, F=0.7, eps=0.1), p.with_(precision="fp32")]
    us = [dev(u), dev(inputs.smooth_state(31, 11, 0.05, 7)), dev(u)]
    single = [host(api.residual(q, v)) for q, v in zip(probs, us)]
    batched = [host(e) for e in api.residual_batched(probs, us)]
    for a, b in zip(single, batched):
        assert np.array_equal(a, b)


def test_wide_meshes_are_refused_where_a_preconditioner_is_needed():
    """Beyond N = 1024 the residual, JVP and zeta work, but the preconditioner (its
    apply holds a block row in LDS) and therefore a solve refuse the mesh."""
    p = api.Problem(1100, 5, -20.0, 20.0, 2.0, F=0.7, eps=0.2)
    with pytest.raises(Exception, match="1024"):
        api.Preconditioner(p, 1)
    with pytest.raises(Exception, match="1024"):
        api.solve(p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM)


def test_fp32_flat_state_without_source_is_exactly_zero():
    p = gprob(inputs.W31X11, eps=0.0, precision="fp32")
    E = gpu_residual(p, inputs.flat_state(p.N, p.M))
    assert np.all(E == 0.0)


def test_jvp_matches_oracle_difference_quotient_and_exact_derivative():
    p = gprob(SMALL_CASES[0][1])
    op = oprob(p)
    u = inputs.smooth_state(p.N, p.M, 0.05, 7)
    z = np.random.default_rng(8).standard_normal(u.size)
    ud, zd = dev(u), dev(z)
    Eu = api.residual(p, ud)
    h = 1e-5
    J = host(api.jvp(p, ud, Eu, zd, h=h))
    Jo = jvp_fd(op, u, oresidual(op, u), z, h)
    sc = row_scale(op, u)
    assert (np.abs(J - Jo) / sc).max() <= 4 * TOL64 / h
    ex = jvp_complex(op, u, z)
    Ja = host(api.jvp(p, ud, Eu, zd, h=0.0))
    rel = np.abs(Ja - ex).max() / np.abs(ex).max()
    log(f"jvp auto-h vs exact: {rel:.2e}")
    assert rel <= 1e-5
    zero = host(api.jvp(p, ud, Eu, torch.zeros_like(zd), h=0.0))
    assert np.all(zero == 0.0)


@pytest.mark.parametrize("cfg", [inputs.W31X11, inputs.W181X61,
                                 dict(N=130, M=7, x1=-10.0, xN=8.0, yM=3.0, F=0.8, eps=0.1)])
def test_zeta_matches_trapezoid_integration(cfg):
    """One wavefront per row: 31 columns (one point per lane), 181 (three per lane) and
    130 (three per lane, the last lanes partly or wholly empty)."""
    p = gprob(cfg)
    u = inputs.smooth_state(p.N, p.M, 0.05, 9)
    z = host(api.zeta(p, dev(u)))
    ref = zeta_grid(oprob(p), u).ravel()
    assert np.abs(z - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_invalid_arguments_are_rejected():
    p = gprob(inputs.W31X11)
    u = dev(inputs.flat_state(p.N, p.M))
    with pytest.raises(Exception):
        api.residual(p.with_(N=3), dev(inputs.flat_state(3, p.M)))
    with pytest.raises(Exception):
        api.residual(p.with_(F=0.0), u)
    with pytest.raises(Exception):
        api.residual(p.with_(N=30, weights="simpson"), dev(inputs.flat_state(30, p.M)))
