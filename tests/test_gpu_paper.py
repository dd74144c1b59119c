"""The paper's own workload (results section: eps = 1, F = 0.7) and the pieces of its
preconditioner study, on the GPU through the C ABI, against the FP64 oracle.

  * 91 x 31 (spacing 0.3, x_1 = -9): the eps = 1 root reached by continuation in steps
    of 0.1 from the flat surface (the bootstrapping paragraph of the JFNK overview),
    against the oracle's root on the same path (stored by tests/golden/make_golden.py
    with its SHA-256): zeta element by element within 1e-8;
  * 361 x 121 on the paper's domain: the eps = 1 root by the same continuation satisfies
    the oracle's E on sampled rows;
  * 45 x 13 (spacing 0.4, x_1 = -9, eps = 1, F = 0.7, flat state; the spectrum figures):
    Jacobian columns from GPU difference quotients against the oracle's exact
    (complex-step) columns, and the preconditioned spectrum with the full linear
    Jacobian clustered about 1.
"""
import hashlib
import os

import numpy as np
import pytest

from oracle import Problem as OProblem
from oracle.equations import residual_rows, zeta_grid
from oracle.solve import jvp_complex
from paper_1403_5044_amd import api, inputs

from gpu_common import dev, gprob, host, log, oprob

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS_PATH = [0.1 * k for k in range(1, 11)]   # the oracle's continuation path, value for value


def _golden(name):
    path = os.path.join(GOLDEN, name)
    want = open(path + ".sha256").read().split()[0]
    assert hashlib.sha256(open(path, "rb").read()).hexdigest() == want
    return np.load(path, allow_pickle=False)


def _continue(cfg, q, tol, prec="fp64", **kw):
    P = api.Preconditioner(gprob(cfg), q)
    u = None
    for e in EPS_PATH:
        un, z, info = api.solve(cfg["F"], e, cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"],
                                precision=prec, precond=P, u0=u, tol=tol, **kw)
        log(f"{cfg['N']}x{cfg['M']} eps {e:.1f}: {info}")
        assert info.status == 0, f"continuation stopped at eps {e}"
        u = un
    P.close()
    return u, z, info


def test_eps1_root_on_91x31_matches_the_oracle_root():
    cfg = dict(N=91, M=31, **inputs.TABLE1[(91, 31)], F=0.7, eps=1.0)
    uo = _golden("table1_91x31_eps1_root.npy")
    zo = zeta_grid(oprob(gprob(cfg)), uo).ravel()
    u, z, info = _continue(cfg, cfg["M"] - 1, 1e-12, max_newton=30)
    dz = np.abs(host(z) - zo).max()
    log(f"91x31 eps=1: zeta vs oracle root {dz:.2e} (max zeta {zo.max():.4f})")
    assert dz <= 1e-8
    assert zo.max() <= cfg["F"] ** 2 / 2
    # the mixed-precision path to the same root, within the stated 1e-6
    um, zm, im = _continue(cfg, cfg["M"] - 1, 1e-10, prec="fp32", max_newton=30)
    dzm = np.abs(host(zm) - zo).max()
    log(f"91x31 eps=1 mixed: zeta vs oracle root {dzm:.2e}")
    assert dzm <= 1e-6


def test_eps1_root_on_361x121_satisfies_the_oracle():
    cfg = dict(inputs.W361X121, eps=1.0)
    u, z, info = _continue(cfg, 8, 1e-10, max_gmres=600, gmres_restart=60, max_newton=20)
    op = OProblem(cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"], F=cfg["F"], eps=1.0)
    NM = op.N * op.M
    rng = np.random.default_rng(11)
    e2 = NM + rng.integers(0, op.M, 32) * op.N + rng.integers(1, op.N, 32)
    rows = np.unique(np.concatenate([np.arange(0, NM, 7), e2]))
    E, _ = residual_rows(op, host(u), rows)
    err = np.abs(E).max()
    zz = host(z)
    log(f"361x121 eps=1: oracle |E| on {rows.size} sampled rows {err:.2e}; "
        f"zeta in [{zz.min():.4f}, {zz.max():.4f}]")
    assert err <= 1e-9
    assert zz.max() <= cfg["F"] ** 2 / 2


def _spectrum_case():
    N, M = 45, 13
    return dict(N=N, M=M, x1=-9.0, xN=-9.0 + 0.4 * (N - 1), yM=0.4 * (M - 1), F=0.7, eps=1.0)


def test_jvp_columns_match_the_oracle_exact_jacobian_on_45x13():
    """Columns of J(u_0) from the GPU's first-order difference quotient against exact
    complex-step columns of the oracle.  The quotient's error is (h/2) z'E''z + O(h^2)
    plus rounding of order macheps |E| / h.  With steps h and h/2 the error must halve
    (a quotient of the wrong function would leave an error that does not go with h),
    and the Richardson combination 2 J(h/2) - J(h), which cancels the first-order
    term, must be at least 20 times closer to the exact column than J(h) (the next
    term is O(h^2)).  The automatic step (about 1e-6 here, 40 times smaller than h)
    must do better than h by a wide margin."""
    cfg = _spectrum_case()
    p = gprob(cfg)
    op = oprob(p)
    n = p.n_unknowns
    u0 = inputs.flat_state(p.N, p.M)
    ud = dev(u0)
    Eu = api.residual(p, ud)
    rng = np.random.default_rng(5)
    cols = np.unique(np.concatenate([[0, n // 2 - 1, n // 2, n - 1], rng.choice(n, 60)]))
    h = 4e-5
    e_h = e_h2 = e_r = e_auto = 0.0
    for i in cols:
        e = np.zeros(n)
        e[i] = 1.0
        ed = dev(e)
        jo = jvp_complex(op, u0, e)
        sc = max(1.0, np.abs(jo).max())
        j1 = host(api.jvp(p, ud, Eu, ed, h=h))
        j2 = host(api.jvp(p, ud, Eu, ed, h=h / 2))
        ja = host(api.jvp(p, ud, Eu, ed))
        e_h = max(e_h, np.abs(j1 - jo).max() / sc)
        e_h2 = max(e_h2, np.abs(j2 - jo).max() / sc)
        e_r = max(e_r, np.abs(2.0 * j2 - j1 - jo).max() / sc)
        e_auto = max(e_auto, np.abs(ja - jo).max() / sc)
    log(f"45x13 JVP columns vs exact over {cols.size} columns: h={h:g} {e_h:.2e}, "
        f"h/2 {e_h2:.2e}, Richardson {e_r:.2e}, automatic h {e_auto:.2e}")
    assert 1.6 <= e_h / e_h2 <= 2.5
    assert e_r <= e_h / 20
    assert e_auto <= 0.1 * e_h   # a step about 40 times smaller than h


def test_full_linear_preconditioner_clusters_the_spectrum_on_45x13():
    """With P the full linear Jacobian, J(u_0) P^-1 = I + eps J_src P^-1 at the flat
    state; its eigenvalues sit in a tight cluster about 1 (the spectrum figure), while
    those of J itself spread over several orders of magnitude.  Gate 0.15 on the
    largest |lambda - 1| (0.10 measured; a banded P with b = 5 already leaves 0.21)."""
    cfg = _spectrum_case()
    p = gprob(cfg)
    n = p.n_unknowns
    ud = dev(inputs.flat_state(p.N, p.M))
    Eu = api.residual(p, ud)
    J = np.empty((n, n))
    Pi = np.empty((n, n))
    P = api.Preconditioner(p, p.M - 1)
    e = np.zeros(n)
    for i in range(n):
        e[:] = 0.0
        e[i] = 1.0
        ed = dev(e)
        J[:, i] = host(api.jvp(p, ud, Eu, ed))
        Pi[:, i] = host(P.apply(ed))
    P.close()
    lam = np.linalg.eigvals(J @ Pi)
    mu = np.linalg.eigvals(J)
    d = np.abs(lam - 1.0)
    log(f"45x13 sigma(J P^-1): max |lambda - 1| {d.max():.3e}; sigma(J): |lambda| in "
        f"[{np.abs(mu).min():.3e}, {np.abs(mu).max():.3e}]")
    assert d.max() <= 0.15
    assert np.abs(mu).max() / np.abs(mu).min() > 10.0
