"""Preconditioner apply and Newton-Krylov solve on the GPU against the oracle."""
import numpy as np
import pytest
import torch

from oracle import flat_state as oflat
from oracle import linear as OL
from oracle.equations import residual_rows, row_scale, zeta_grid
from oracle.equations import residual as oresidual
from oracle.solve import newton
from paper_1403_5044_amd import api, inputs

from gpu_common import dev, gprob, host, log, oprob

pytestmark = pytest.mark.gpu

TINY = dict(N=9, M=5, x1=-3.0, xN=3.0, yM=2.0, F=0.7, eps=0.3)


def _backward_error(P, x, b):
    """Normwise backward error ||P x - b||_inf / (||P||_inf ||x||_inf + ||b||_inf)."""
    r = P @ x - b
    return np.abs(r).max() / (np.abs(P).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())
SMALL = dict(N=15, M=7, x1=-6.0, xN=6.0, yM=5.0, F=0.7, eps=0.05)


@pytest.mark.parametrize("cfg", [TINY, SMALL, inputs.W31X11,
                                 dict(N=41, M=13, x1=-8.0, xN=8.0, yM=6.0, F=0.9, eps=0.1,
                                      weights="simpson")])
def test_preconditioner_apply_matches_dense_solve(cfg):
    p = gprob(cfg)
    op = oprob(p)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(p.n_unknowns)
    for q in sorted({0, 1, 2, p.M - 1}):
        pre_o = OL.BlockPreconditioner(op, q)
        Pm = pre_o.matrix()
        P = api.Preconditioner(p, q)
        x = host(P.apply(dev(b)))
        P.close()
        res = _backward_error(Pm, x, b)
        xo = pre_o.solve(b)
        rel = np.abs(x - xo).max() / np.abs(xo).max()
        log(f"N={p.N} M={p.M} q={q}: backward err {res:.2e}, vs oracle {rel:.2e}")
        assert res <= 1e-12  # normwise backward error, ~4 n eps at n = 2410
        assert rel <= 1e-8


def test_preconditioner_apply_in_place():
    p = gprob(inputs.W31X11)
    b = np.random.default_rng(1).standard_normal(p.n_unknowns)
    P = api.Preconditioner(p, 1)
    x1 = host(P.apply(dev(b)))
    bd = dev(b)
    P.apply(bd, out=bd)
    assert np.array_equal(host(bd), x1)
    P.close()


def test_batched_apply_is_bitwise_the_single_apply():
    """Several preconditioners applied in shared launches give the bits of one apply each:
    super-row handles of different widths in one round, a handle used twice (second
    round), q = 0 and a one-block-row band (N = 700) through the single path, an
    in-place request, and 33 distinct handles (a full round of 32, then a round of 1)."""
    dom = dict(x1=-16.0, xN=8.0, yM=12.0)
    pcs = [api.Preconditioner(api.Problem(61, 21, **dom, F=0.7, eps=0.1), 3),
           api.Preconditioner(api.Problem(121, 41, **dom, F=0.9, eps=0.1), 5),
           api.Preconditioner(api.Problem(31, 11, -8.0, 8.0, 8.0, F=0.6, eps=0.1), 0),
           api.Preconditioner(api.Problem(700, 9, -14.0, 40.0, 6.0, F=0.7, eps=0.1), 2),
           api.Preconditioner(api.Problem(41, 13, -8.0, 8.0, 6.0, F=0.9, eps=0.1,
                                          weights="simpson"), 2)]
    small = [api.Preconditioner(api.Problem(13, 5, -4.0, 4.0, 3.0, F=0.5 + 0.02 * k,
                                            eps=0.1), 1 + k % 3) for k in range(33)]
    rng = np.random.default_rng(11)
    for reqs in ([0, 1, 0, 2, 3, 4, 1], list(range(len(pcs), len(pcs) + 33))):
        allp = pcs + small
        sel = [allp[i] for i in reqs]
        bs = [dev(rng.standard_normal(P.prob.n_unknowns)) for P in sel]
        single = [host(P.apply(b)) for P, b in zip(sel, bs)]
        outs = [torch.empty_like(b) for b in bs]
        outs[-1] = bs[-1].clone()
        bs[-1] = outs[-1]  # in place
        got = [host(x) for x in api.Preconditioner.apply_batched(sel, bs, outs)]
        for i, (a, g) in enumerate(zip(single, got)):
            assert np.array_equal(a, g), (reqs[i], sel[i].prob.N, sel[i].prob.M, sel[i].q)
        log(f"batched apply of {len(sel)} requests: bitwise equal")
    for P in pcs + small:
        P.close()


def _oracle_root(p, tol=1e-12):
    op = oprob(p)
    u, info = newton(op, oflat(op), tol=tol)
    assert info.converged
    return u


@pytest.mark.parametrize("q", [0, 1, 10])
def test_31x11_fp64_solve_matches_oracle_root(q):
    p = gprob(inputs.W31X11)
    uo = _oracle_root(p)
    u, z, info = api.solve(p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM, q_blocks=q, tol=1e-11)
    log(f"31x11 q={q}: {info}")
    assert info.status == 0
    ug = host(u)
    zg = host(z)
    zo = zeta_grid(oprob(p), uo).ravel()
    assert np.abs(zg - zo).max() <= 1e-8
    assert np.abs(ug - uo).max() <= 1e-7
    assert np.abs(oresidual(oprob(p), ug)).max() <= 2e-11
    assert zg.max() <= p.F ** 2 / 2


def test_31x11_mixed_precision_solve_within_stated_bound():
    p = gprob(inputs.W31X11)
    uo = _oracle_root(p)
    u, z, info = api.solve(p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM, precision="fp32",
                           tol=1e-10)
    log(f"31x11 mixed: {info}")
    assert info.status == 0
    zo = zeta_grid(oprob(p), uo).ravel()
    err = np.abs(host(z) - zo).max()
    log(f"31x11 mixed zeta err {err:.2e}")
    assert err <= 1e-6


def test_solve_continuation_from_caller_state():
    p = gprob(inputs.W31X11)
    u, _, info = api.solve(p.F, 0.05, p.N, p.M, p.x1, p.xN, p.yM)
    assert info.status == 0
    u2, z2, info2 = api.solve(p.F, 0.1, p.N, p.M, p.x1, p.xN, p.yM, u0=u)
    assert info2.status == 0
    uo = _oracle_root(p.with_(eps=0.1))
    zo = zeta_grid(oprob(p.with_(eps=0.1)), uo).ravel()
    assert np.abs(host(z2) - zo).max() <= 1e-8


def test_181x61_solve_is_a_root_of_the_oracle_system():
    """181 x 61, eps 0.1: the GPU root, checked by the oracle on
    every E1/E4/E6 entry and on sampled E2 entries; FP32-mixed root agrees."""
    p = gprob(inputs.W181X61)
    u, z, info = api.solve(p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM, tol=1e-10)
    log(f"181x61 fp64: {info}")
    assert info.status == 0
    ug = host(u)
    op = oprob(p)
    NM = p.N * p.M
    rng = np.random.default_rng(0)
    e2 = NM + rng.integers(0, p.M, 40) * p.N + rng.integers(1, p.N, 40)
    rows = np.unique(np.concatenate([np.arange(NM), e2]))
    Eo, _ = residual_rows(op, ug, rows)
    log(f"181x61 oracle |E(u_gpu)| max {np.abs(Eo).max():.2e}")
    assert np.abs(Eo).max() <= 1e-9
    zg = host(z)
    assert zg.max() <= p.F ** 2 / 2
    um, zm, infom = api.solve(p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM, precision="fp32",
                              tol=1e-10)
    log(f"181x61 mixed: {infom}")
    assert infom.status == 0
    err = np.abs(host(zm) - zg).max()
    log(f"181x61 mixed vs fp64 zeta {err:.2e}")
    assert err <= 1e-6


def test_preconditioner_graph_replays_match_the_dense_solve():
    """The band substitution is replayed from a captured graph: apply several
    times with other GPU work and synchronisations in between, each result
    checked against the dense solve and repeats checked bitwise."""
    p = gprob(dict(N=41, M=13, x1=-8.0, xN=8.0, yM=6.0, F=0.8, eps=0.1))
    op = oprob(p)
    P = api.Preconditioner(p, 3)
    Pm = OL.BlockPreconditioner(op, 3).matrix()
    rng = np.random.default_rng(12)
    first = {}
    for rep in range(4):
        for k in range(3):
            b = np.random.default_rng(100 + k).standard_normal(p.n_unknowns)
            x = host(P.apply(dev(b)))
            res = _backward_error(Pm, x, b)
            assert res <= 1e-12, (rep, k, res)
            if rep == 0:
                first[k] = x
            else:
                assert np.array_equal(first[k], x)
            api.residual(p, dev(inputs.smooth_state(p.N, p.M, 0.05, rep)))
            torch.cuda.synchronize()
        _ = rng.standard_normal(3)
    P.close()


@pytest.mark.parametrize("N,M", [(64, 6), (65, 7), (121, 9), (181, 7), (182, 5), (183, 5),
                                 (192, 5), (241, 5), (256, 4), (257, 4), (512, 4), (521, 4),
                                 (667, 4), (721, 4), (768, 4), (769, 4), (1024, 4)])
def test_preconditioner_wide_blocks_match_dense_solve(N, M):
    """Every diagonal-block inversion variant against the oracle's dense P: the
    register-tile kernel with 1, 2 and 3 panel rows per lane (13- and 14-row tiles on
    either side of N = 182), the column-strip launches up to N = 256, and beyond that
    the panel and update launches with 2 and 4 panel rows per thread.  From N = 667 the
    substitution runs one block row per step (no super rows), the path of 721 x 241;
    N = 1024 is the largest mesh width that a preconditioner accepts."""
    p = api.Problem(N, M, -10.0, 8.0, 3.0, F=0.75, eps=0.1)
    op = oprob(p)
    b = np.random.default_rng(N).standard_normal(p.n_unknowns)
    for q in (0, 1, M - 1):
        Pm = OL.BlockPreconditioner(op, q).matrix()
        P = api.Preconditioner(p, q)
        x = host(P.apply(dev(b)))
        P.close()
        res = _backward_error(Pm, x, b)
        log(f"N={N} M={M} q={q}: backward err {res:.2e}")
        assert res <= 1e-12  # normwise backward error, ~4 n eps at n = 2410


@pytest.mark.parametrize("N,M,q", [(31, 40, 8), (31, 60, 10), (15, 20, 19), (41, 13, 6),
                                   (41, 14, 3), (21, 9, 2), (300, 14, 4), (700, 9, 2)])
def test_preconditioner_band_orders_match_dense_solve(N, M, q):
    """The band is eliminated from both ends with q separator rows last.  Cases: a top and
    a bottom super row too large to share a launch (31 x 40, q = 8), a separator super row
    that has to shrink to fit (31 x 60, q = 10), q = M - 1 (no bottom chain), and M - q
    odd and even (chains of equal and unequal length).  With N > 256 each eliminated
    row's Schur updates run as one row product: at 300 x 14 (q = 4) and 700 x 9 (q = 2)
    the chains meet, so the products leave out the next diagonal blocks and the bottom
    updates that wait for the top chain's, which run in launches of their own; 700 also
    substitutes one block row per step."""
    p = api.Problem(N, M, -10.0, 8.0, 3.0, F=0.75, eps=0.1)
    op = oprob(p)
    Pm = OL.BlockPreconditioner(op, q).matrix()
    P = api.Preconditioner(p, q)
    for k in range(2):
        b = np.random.default_rng(1000 * N + M + k).standard_normal(p.n_unknowns)
        x = host(P.apply(dev(b)))
        res = _backward_error(Pm, x, b)
        log(f"N={N} M={M} q={q} rhs {k}: backward err {res:.2e}")
        assert res <= 1e-12
    P.close()


@pytest.mark.parametrize("cfg,q", [(inputs.W181X61, 5), (dict(N=241, M=21, x1=-16.0, xN=8.0,
                                                              yM=12.0, F=0.8, eps=0.2), 8)])
def test_cold_solve_equals_prebuilt_preconditioner_bitwise(cfg, q):
    """A cold solve builds its preconditioner on a helper stream beside the first residual
    evaluation, and the band factorisation runs the super-row operators on another helper
    stream.  The set-up is deterministic, so the cold solve must equal, bit for bit, the
    same solve with the preconditioner built beforehand by the public call; a missing
    ordering between the streams would show up as a difference."""
    p = gprob(cfg)
    args = (p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM)
    u1, z1, i1 = api.solve(*args, q_blocks=q, tol=1e-10)
    P = api.Preconditioner(p, q)
    u2, z2, i2 = api.solve(*args, precond=P, tol=1e-10)
    P.close()
    u3, z3, i3 = api.solve(*args, q_blocks=q, tol=1e-10)
    log(f"{p.N}x{p.M} q={q}: cold {i1}, prebuilt {i2}")
    assert i1.status == 0 and i2.status == 0 and i3.status == 0
    assert (i1.newton_iters, i1.gmres_iters) == (i2.newton_iters, i2.gmres_iters)
    assert torch.equal(u1, u2) and torch.equal(z1, z2)
    assert torch.equal(u1, u3) and torch.equal(z1, z3)
