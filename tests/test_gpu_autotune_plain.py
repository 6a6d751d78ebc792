"""The plain-step autotuner (cells per block of the update kernel) on the GPU: every candidate
leaves the state bitwise identical, the state is restored, and the chosen shape is applied."""
import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I
from tests.gpu_util import HAVE_GPU, banner, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_1908_01682_amd import autotune as A
    from paper_1908_01682_amd import tfsph as T


def _state(sim):
    """The fields a step writes (the dust density is a diagnostic the step leaves alone)."""
    out = {}
    for tag, ph in (("g", sim.gas), ("d", sim.dust)):
        for k, v in ph.numpy().items():
            if v is not None and not (tag == "d" and k == "rho"):
                out[tag + k] = np.ascontiguousarray(v).tobytes()
    return out


@pytest.mark.parametrize("name,make", [
    ("box3d", lambda: I.dusty_box(n_side=32, cells_per_axis=16, regions_per_axis=4)),
    ("wave2d", lambda: I.wave_2d(n_side=64, amp=1e-2)),
    ("shock1d", lambda: I.dusty_shock(n=4000)),
])
def test_tune_plain_is_bitwise_neutral(tmp_path, name, make):
    prob = make()
    banner(f"tune_plain {name} n=({prob.gas.n},{prob.dust.n})")
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    before = _state(sim)
    res = A.tune_plain(sim, steps=5, use_cache=False, path=str(tmp_path / "c.json"))
    assert res["bitwise_identical"] and res["cells_per_block"] in A.CANDIDATE_CELLS_PER_BLOCK
    after = _state(sim)
    assert before == after
    sim.step(3)
    torch.cuda.synchronize()
    tuned = _state(sim)
    sim.close()
    ref = T.Simulation(prob, precision=T.TFSPH_F32)
    ref.step(3)
    torch.cuda.synchronize()
    plain = _state(ref)
    ref.close()
    assert tuned == plain
    # a second call finds the cache
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    hit = A.tune_plain(sim, steps=5, path=str(tmp_path / "c.json"))
    sim.close()
    assert hit["cached"] and hit["cells_per_block"] == res["cells_per_block"]
