"""What the trained controller gains over the plain rule (GPU).

The perceptron is trained on the GPU (the library's forward, backward and Adam
kernels) with samples the method generates itself: per-block errors of
emulated builds at s = 1..8 along two synthetic SCF sequences.  On a held-out
sequence the controlled run must use fewer digit products than the plain rule
in total, never more in any iteration, and stay at the plain rule's accuracy
(K error within a small factor of the plain rule's, energies as close to
FP64)."""
import numpy as np
import pytest

import dfinputs

pytestmark = pytest.mark.gpu

NAO, NAUX, NOCC, NITER = 128, 512, 16, 8


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _sequence(torch, seed):
    p = dfinputs.make_problem(nao=NAO, naux=NAUX, nocc=NOCC, L=16.0, seed=seed, block_scale=4)
    orbs = dfinputs.perturbed_orbitals(p["C"], NITER, seed=seed, eps_hi=1e-2, eps_lo=1e-8)
    B = torch.from_numpy(p["B"]).cuda()
    return B, [torch.from_numpy(c).cuda() for c in orbs]


def test_trained_controller_beats_plain_rule(torch_dev):
    torch = torch_dev
    from paper_2601_08077_amd import Context, adaptive, controller
    ctx = Context()
    xs, ts, ms = [], [], []
    for seed in (1, 2):
        B, orbs = _sequence(torch, seed)
        be = torch.empty(NAUX * NAO, dtype=torch.int32, device="cuda")
        ctx.df_b_exponents(B, be)
        x, t, m = controller.collect_samples(ctx, B, be, orbs)
        xs.append(x), ts.append(t), ms.append(m)
    x, t, m = np.concatenate(xs), np.concatenate(ts), np.concatenate(ms)
    assert x.shape == (2 * NITER * NAUX // 64, 16) and m.sum() > 0.9 * m.size
    params, losses = controller.train(ctx, x, t, m, steps=1500, batch=128, lr=3e-3, seed=0)
    assert losses[-50:].mean() < 0.1 * losses[:10].mean()
    rms = controller.evaluate(ctx, params, x, t, m)
    print(f"training rms error {rms:.3f} decades, loss {losses[0]:.3g} -> {losses[-1]:.3g}")
    assert rms < 1.0

    B, orbs = _sequence(torch, 3)
    be = torch.empty(NAUX * NAO, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be)
    ctx.df_set_block_precision(None)
    ctx.df_set_pblk(64)
    ctx.ensure_workspace(NAUX, NAO, NOCC)
    plain = adaptive.run_sequence(ctx, B, be, orbs, fp64_check=True)
    ctl = controller.run_controlled(ctx, B, be, orbs, params, fp64_check=True, spot=2)
    nb = NAUX // 64
    w_plain = sum(nb * r["slices"] * (r["slices"] + 1) // 2 for r in plain)
    w_ctl = sum(r["work"] for r in ctl)
    for a, c in zip(plain, ctl):
        print(f"it {a['iteration']} plain s={a['slices']} err={a['k_maxabs_rel_fro']:.2e} | "
              f"ctl {c['slices']} work {c['work']}/{c['work_ref']} err={c['k_maxabs_rel_fro']:.2e}"
              f" fb={c['fallback']}")
        assert c["work"] <= c["work_ref"] or c["fallback"]
        if c["s_ref"] == a["slices"]:
            assert c["k_maxabs_rel_fro"] <= 4.0 * a["k_maxabs_rel_fro"] + 1e-15
    print(f"digit products: controller {w_ctl} vs plain {w_plain}")
    assert w_ctl < 0.9 * w_plain
    assert abs(ctl[-1]["energy_err"]) <= 4.0 * abs(plain[-1]["energy_err"]) + 1e-12
    ctx.close()


def test_trained_controller_beats_plain_rule_in_time(torch_dev):
    """The controller benchmark's sequence at its shape (nao 1536, naux 6144,
    nocc 192, 30 iterations) with a training set of about 20k samples: the
    controlled run (features, prediction, per-block builds, FP64 spot checks
    and any fallback rebuilds, all inside the timed region) takes less GPU
    time than the plain rule's at the same reference counts, with a largest K
    error no worse than the plain rule's."""
    import argparse
    import bench
    args = argparse.Namespace(ctl_samples=20000, ctl_train_steps=8000, ctl_nao=1536,
                              ctl_slack=0.5, ctl_min_gain=0.1)
    out = bench.controller_workload(args)
    print(f"time: controller {out['controller_total_ms']:.1f} ms vs plain "
          f"{out['plain_total_ms']:.1f} ms ({out['speedup_vs_plain']:.3f}x); max K error "
          f"{out['max_k_err_controller']:.2e} vs {out['max_k_err_plain']:.2e}; "
          f"{out['controller_iterations']} controlled iterations, {out['fallbacks']} fallbacks")
    assert out["controller_iterations"] > 0
    assert out["controller_total_ms"] < out["plain_total_ms"]
    assert out["max_k_err_controller"] <= out["max_k_err_plain"]
