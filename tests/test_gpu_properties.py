"""Property tests on the GPU: random compiled sizes (radices 2, 3 and 5), random
boxes, random Gaussian mixtures and all three precisions, each solve against
the oracle's on the same input at the stated tolerance.

The cases come from hypothesis with derandomize=True, so every run draws the
same cases (a GPU test must be repeatable); widening max_examples widens the
search.  The oracle builds its own kernel spectrum for every box, so a case
costs about a second of host time.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle as O
import workloads as W
from gpu_common import TOL, max_rel, torch_cuda

pytestmark = pytest.mark.gpu
psn = pytest.importorskip("paper_1612_01799_amd")

SIZES = [8, 12, 16, 24, 32, 48, 64, 96]
SETTINGS = settings(max_examples=25, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@st.composite
def boxes(draw, per_axis):
    """A box with a lower corner in [-3, -0.5] and edges in [1, 6] per axis,
    n points per axis (or n_q per axis), and a mixture of 1-4 Gaussians
    inside its middle, widths a fraction of the shortest half-edge."""
    n0 = draw(st.sampled_from(SIZES))
    n3 = tuple(draw(st.sampled_from(SIZES)) for _ in range(3)) if per_axis else (n0,) * 3
    a = tuple(draw(st.floats(-3.0, -0.5)) for _ in range(3))
    b = tuple(a[q] + draw(st.floats(1.0, 6.0)) for q in range(3))
    k = draw(st.integers(1, 4))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    dt = draw(st.sampled_from(["f64", "f32", "split"]))
    return n3, a, b, k, seed, dt


def _check(n3, a, b, k, seed, dt):
    torch = torch_cuda()
    box = W.Box(a, b, n3)
    half = min(0.5 * (b[q] - a[q]) for q in range(3))
    mix = W.draw_mixture(seed, k, -0.3 * half, 0.3 * half, 0.12 * half, 0.3 * half, 0.5, 1.5, box)
    mix.centres = mix.centres + np.asarray(box.centre())[None, :]
    rho = W.mixture_density(mix)
    ref = O.solve(rho, O.half_spectrum(O.kernel_spectrum(box, 1e-12)))
    n = n3 if len(set(n3)) > 1 else n3[0]
    print(f"property case: n={n3} box={a}..{b} k={k} seed={seed} {dt}", flush=True)
    plan = psn.Plan(n, box=(a, b), tol=1e-12, dtype=dt).build()
    u = plan.solve(torch.from_numpy(rho).to("cuda", plan.io_dtype()))
    torch.cuda.synchronize()
    err = max_rel(u.double().cpu().numpy(), ref)
    assert err <= TOL[dt], (n3, a, b, k, seed, dt, err)


@SETTINGS
@given(boxes(per_axis=False))
def test_random_cube_grids_match_oracle(case):
    _check(*case)


@SETTINGS
@given(boxes(per_axis=True))
def test_random_per_axis_grids_match_oracle(case):
    _check(*case)
