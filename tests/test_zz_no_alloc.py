"""The residual entry point that allocates nothing (shipwave_residual_noalloc), through
the C ABI, against shipwave_residual: two calls in a row on the library's fixed array,
the second with a smaller mesh, each within the FP64 parity gate (1e-11 of the summed
term magnitudes) of the allocating entry point; the FP32 path within the FP32 bound; and
an oversized mesh rejected on the host before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import residual as oresidual
from oracle.equations import row_scale
from paper_1403_5044_amd import _lib, api, inputs

from gpu_common import dev, gprob, host, log, oprob

pytestmark = pytest.mark.gpu


def _pair(p, u):
    ud = dev(u)
    ref = host(api.residual(p, ud))
    out = torch.full_like(ud, float("nan"))
    got = host(api.residual_noalloc(p, ud, out))
    return ref, got


def test_noalloc_matches_the_allocating_entry_point_twice_then_smaller():
    cases = [(gprob(inputs.W181X61), inputs.batch_181x61(2)[1]),
             (gprob(inputs.W31X11), inputs.smooth_state(31, 11, 0.05, 3))]
    for p, u in cases:
        ref, got = _pair(p, u)
        sc = row_scale(oprob(p), u)
        err = (np.abs(got - ref) / sc).max()
        log(f"{p.N}x{p.M} fp64: noalloc vs shipwave_residual {err:.2e}")
        assert np.all(np.isfinite(got))
        assert err <= 1e-11
        # and against the oracle itself
        assert (np.abs(got - oresidual(oprob(p), u)) / sc).max() <= 1e-11


def test_noalloc_fp32_and_repeat():
    p = gprob(inputs.W181X61, precision="fp32")
    u = inputs.batch_181x61(1)[0]
    ref, got = _pair(p, u)
    sc = row_scale(oprob(p), u)
    err = (np.abs(got - ref) / sc).max()
    log(f"181x61 fp32: noalloc vs shipwave_residual {err:.2e}")
    assert err <= 2.0 ** -19
    _, again = _pair(p, u)
    assert np.array_equal(got, again)


def test_noalloc_rejects_a_mesh_beyond_the_fixed_array():
    p = api.Problem(1024, 300, -14.0, 40.0, 18.0, F=0.7, eps=0.1, precision="fp32")
    u = torch.zeros(p.n_unknowns, dtype=torch.float64, device="cuda")
    E = torch.zeros_like(u)
    with pytest.raises(_lib.ShipwaveError) as ei:
        api.residual_noalloc(p, u, E)
    assert ei.value.code == -2
    torch.cuda.synchronize()
    assert torch.all(E == 0)
