"""Learned reflection probabilities on the GPU (Methods): the score-function
gradient of gwg_omega_gradient against the oracle's estimator on the same
paths, and a short pre-optimisation that raises the eyebox throughput."""
import numpy as np
import pytest
import torch

import inputs
import paper_2601_04370_amd as gwg
from paper_2601_04370_amd import optim

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,kw", [
    ("plain_fp64", dict(rays_per_point=3000)),
    ("diff_1200", dict(rays_per_point=64, fov_n=3)),
    ("batched", dict(n_designs=2, rays_per_point=40, fov_n=3, lambdas_nm=(420.0, 680.0))),
])
@pytest.mark.parametrize("weights", ["ones", "random"])
def test_omega_gradient_matches_oracle(gctx, orc, name, kw, weights):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    _, counts, _, _, _ = gctx.trace_forward(scene, thk, w.seed, 0, 0)
    rng = np.random.default_rng(2)
    W = np.ones(scene.shape) if weights == "ones" else rng.uniform(-1.0, 2.0, scene.shape)
    g = gctx.omega_gradient(torch.tensor(W), counts, scene).cpu().numpy()
    osc = orc.OracleScene(w, inp)
    og, _ = orc.omega_score_gradient(osc, W, counts.cpu().numpy())
    print(f"  {name}: gpu {g} oracle {og}", flush=True)
    assert np.allclose(g, og, rtol=1e-11, atol=1e-13 * np.abs(og).max())
    # deterministic
    g2 = gctx.omega_gradient(torch.tensor(W), counts, scene).cpu().numpy()
    assert np.array_equal(g, g2)


def test_learned_omega_raises_throughput(gctx):
    w = inputs.small_variant("plain_fp64", rays_per_point=20000)
    inp = inputs.make_inputs(w)
    scene0 = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")

    def throughput(om):
        sc = gwg.SceneSpec.from_workload(w, {**inp, "omega": om})
        vals = []
        for s in range(3):
            _, c, _, _, _ = gctx.trace_forward(sc, thk, 777 + s, 0, 0)
            vals.append(float(c.sum()) / w.rays_per_point)
        return float(np.mean(vals))

    om0 = np.asarray(inp["omega"], dtype=np.float64)
    om = optim.learn_reflection_probabilities(gctx, w, inp, iters=40, lr=0.2, seed=w.seed)
    t0, t1 = throughput(om0), throughput(om)
    print(f"  omega {om0} -> {om}; throughput {t0:.4f} -> {t1:.4f}", flush=True)
    assert np.all((om >= 0.02) & (om <= 0.98))
    assert t1 > t0 + 0.01
