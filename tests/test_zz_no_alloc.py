"""The no-allocation entry point tfsph_step_noalloc against tfsph_init + tfsph_step, through
the C ABI: same kernels on the library's static workspace, so the states must be bitwise equal.
Two calls in a row, the second on a smaller problem (the static array keeps the first call's
contents), and the flags the call exports against tfsph_get_flags."""
import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I
from tests.gpu_util import HAVE_GPU, banner, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_1908_01682_amd import tfsph as T


def _arrays(ph):
    d = ph.numpy()
    return {k: v for k, v in d.items() if v is not None}


def _run_both(prob, precision, n_steps):
    banner(f"noalloc {prob.name} n=({prob.gas.n},{prob.dust.n}) precision={precision} steps={n_steps}")
    ref = T.Simulation(prob, precision=precision)
    ref.step(n_steps)
    ref_flags = ref.flags()
    st = T.DeviceState(prob, precision=precision)
    flags = torch.full((1,), 0xFFFF, dtype=torch.int32, device="cuda")
    one = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    T.tfsph_step_noalloc(st.params, st.state, n_steps, flags, one)
    torch.cuda.synchronize()
    for name, a, b in (("gas", ref.gas, st.gas), ("dust", ref.dust, st.dust)):
        A, B = _arrays(a), _arrays(b)
        assert A.keys() == B.keys()
        for k in A:
            assert np.array_equal(A[k], B[k]), (name, k)
    got = (int(flags.cpu().numpy()[0]) & 0xFFFFFFFF, int(one.cpu().numpy()[0]))
    ref.close()
    assert got == ref_flags, (got, ref_flags)


def test_noalloc_matches_init_and_step_two_calls():
    """First a 2D wave of 64^2 + 64^2 particles (FP32, 20 steps), then a smaller problem on the
    same static array: a 1D shock tube of 3000 + 3000 particles with viscosity and energy
    (FP32, 15 steps), then an FP64 wave of 200 + 200 with one-phase cells planted."""
    _run_both(I.wave_2d(n_side=64, amp=1e-2), 0, 20)
    _run_both(I.dusty_shock(n=3000, t_stop=1e-3), 0, 15)
    prob = I.dusty_wave(n_side=200, amp=1e-2, cells_per_axis=100)
    prob.dust.x = prob.dust.x[:150]
    prob.dust.v = prob.dust.v[:150]
    prob.dust.m = prob.dust.m[:150]
    prob.dust.id = prob.dust.id[:150]
    _run_both(prob, 1, 7)


def test_noalloc_second_scheme_and_zero_steps():
    """The second-order IMEX step through the same entry point, and n_steps = 0 (the canonical
    ordering of tfsph_init alone)."""
    prob = I.wave_2d(n_side=48, amp=1e-2)
    prob.params = prob.params.replace(scheme=1)
    _run_both(prob, 0, 5)
    _run_both(I.dusty_box(n_side=16, cells_per_axis=8, regions_per_axis=2), 0, 0)


def test_noalloc_rejects_a_problem_beyond_the_static_array():
    """The 3D box of 128^3 + 128^3 particles needs several hundred MB: refused on the host with
    TFSPH_E_WORKSPACE before anything is enqueued."""
    prob = I.dusty_box(n_side=128, cells_per_axis=64)
    st = T.DeviceState(prob, precision=0)
    with pytest.raises(T.TfsphError) as e:
        T.tfsph_step_noalloc(st.params, st.state, 1)
    assert e.value.status == -2
