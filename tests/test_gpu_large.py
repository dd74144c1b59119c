"""361x121 and 721x241 on the paper's domain, on the GPU: the FP64
root satisfies the oracle's E on sampled rows (every E1 row at a stride and E2 rows at
random collocation points, each E2 row a full sum over the grid), and the mixed-precision
root agrees with it within the stated bound."""
import numpy as np
import pytest

from oracle import Problem as OProblem
from oracle.equations import residual_rows
from paper_1403_5044_amd import api, inputs

from gpu_common import host, log

pytestmark = pytest.mark.gpu


def _oracle_E_sampled(cfg, F, eps, u, stride, n_e2):
    op = OProblem(cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"], F=F, eps=eps)
    NM = op.N * op.M
    rng = np.random.default_rng(7)
    e2 = NM + rng.integers(0, op.M, n_e2) * op.N + rng.integers(1, op.N, n_e2)
    rows = np.unique(np.concatenate([np.arange(0, NM, stride), e2]))
    E, _ = residual_rows(op, host(u), rows)
    return np.abs(E).max()


def _solve(cfg, F, eps, prec, P, u0=None):
    return api.solve(F, eps, cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"], precision=prec,
                     precond=P, u0=u0, tol=1e-10, max_gmres=600, gmres_restart=60, max_newton=20)


def test_361x121_root_satisfies_the_oracle_and_mixed_agrees():
    cfg = dict(inputs.W361X121, F=1.0, eps=0.3)
    P = api.Preconditioner(api.Problem(**cfg), 8)
    u64, z64, i64 = _solve(cfg, 1.0, 0.3, "fp64", P)
    u32, z32, i32 = _solve(cfg, 1.0, 0.3, "fp32", P)
    P.close()
    log(f"361x121 F=1 eps=0.3 fp64 {i64}; mixed {i32}")
    assert i64.status == 0 and i32.status == 0
    err = _oracle_E_sampled(inputs.W361X121, 1.0, 0.3, u64, 7, 24)
    dz = np.abs(host(z64) - host(z32)).max()
    log(f"361x121: oracle |E| on sampled rows {err:.2e}; mixed vs fp64 zeta {dz:.2e}")
    assert err <= 1e-9
    assert dz <= 1e-6
    assert host(z64).max() <= cfg["F"] ** 2 / 2


def test_721x241_continuation_step_satisfies_the_oracle():
    cfg = inputs.W721X241
    P = api.Preconditioner(api.Problem(**cfg), inputs.Q_BLOCKS[(cfg["N"], cfg["M"])])
    um, zm, im = _solve(cfg, cfg["F"], 0.1, "fp32", P)
    assert im.status == 0
    u2, z2, i2 = _solve(cfg, cfg["F"], 0.2, "fp32", P, u0=um)
    u64, z64, i64 = _solve(cfg, cfg["F"], 0.2, "fp64", P, u0=um)
    P.close()
    log(f"721x241 eps=0.2 from eps=0.1: mixed {i2}; fp64 {i64}")
    assert i2.status == 0 and i64.status == 0
    err = _oracle_E_sampled(cfg, cfg["F"], 0.2, u64, 97, 8)
    dz = np.abs(host(z64) - host(z2)).max()
    log(f"721x241: oracle |E| on sampled rows {err:.2e}; mixed vs fp64 zeta {dz:.2e}")
    assert err <= 1e-9
    assert dz <= 1e-6
