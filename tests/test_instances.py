"""The counter-based inventory generator of the largest workload: its CPU rows and its
torch fill (run here on the CPU) give the same numbers, and the draws have Poisson
moments."""
import numpy as np
import torch

from paper_2406_01939_amd.instances import PoissonX0, zipf_probs, make_instance


def test_rows_equal_tensor_fill():
    lam = 0.8 * 2e6 * zipf_probs(3000) * 1.5 / 200
    g = PoissonX0(lam, 77)
    out = torch.empty((3000, 200), dtype=torch.int32)
    g.device(5, 200, out, chunk=700)
    np.testing.assert_array_equal(out.numpy(), g.rows(5, np.arange(3000), 200))
    ks = np.array([0, 17, 2999])
    np.testing.assert_array_equal(out.numpy()[ks], g.rows(5, ks, 200))


def test_poisson_moments():
    lam = np.array([0.05, 1.0, 7.5, 300.0, 4000.0])
    g = PoissonX0(lam, 3)
    x = g.rows(0, np.arange(5), 20000).astype(np.float64)
    for k in range(5):
        se = np.sqrt(lam[k] / x.shape[1])
        assert abs(x[k].mean() - lam[k]) < 5 * se + 1e-3, k
        assert abs(x[k].var() / lam[k] - 1.0) < 0.08, k
    # trajectories draw independently
    y = g.rows(1, np.arange(5), 20000)
    assert not np.array_equal(x.astype(np.int32), y)


def test_prefix_instance_keeps_full_scale_inventory():
    inst = make_instance("mlp_batch16_n500_k1e6_t1e7", n_traj=2, T_orders=500, K=5000)
    assert inst.x0 is None and inst.total_orders == 1000
    r = inst.x0_rows(1, [0, 1])
    lam0 = 0.8 * 1e7 * zipf_probs(5000)[0] * inst.qty.mean() / 500
    assert r.shape == (2, 500) and 0.5 * lam0 < r[0].mean() < 2 * lam0
