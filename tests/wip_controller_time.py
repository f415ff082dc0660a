"""Wall-time gain of the trained controller over the plain rule (GPU).  Not
collected until it passes: run it by naming this file."""
import numpy as np
import pytest

import dfinputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _packed_sequence(torch, ctx, nao, seed, n_iter):
    """Packed B (aux blocks ordered by max |B_b|), its exponents and a
    sequence of orbitals; naux 4 nao, nocc nao / 8, per-block scales."""
    from paper_2601_08077_amd import DF_PACKED, controller
    naux, nocc = 4 * nao, nao // 8
    p = dfinputs.make_problem_device(nao=nao, naux=naux, nocc=nocc, L=24.0, seed=seed,
                                     block_scale=4)
    Bp = dfinputs.pack_lower(p["B"])
    del p["B"]
    B, _ = controller.order_aux_blocks(ctx, Bp, 64, DF_PACKED, naux, nao)
    del Bp
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be, layout=DF_PACKED, naux=naux, nao=nao)
    orbs = [torch.from_numpy(c).cuda()
            for c in dfinputs.perturbed_orbitals(p["C_host"], n_iter, seed=seed)]
    return B, be, orbs


def test_trained_controller_beats_plain_rule_in_time(torch_dev):
    """The controller's sequence (features, prediction, per-block builds, FP64
    spot checks and any fallback rebuilds, all inside the timed region) takes
    less GPU time than the plain rule's at the same reference counts, with a
    largest K error no worse than the plain rule's."""
    torch = torch_dev
    from paper_2601_08077_amd import DF_PACKED, Context, adaptive, controller
    ctx = Context()
    ctx.df_set_pblk(64)
    xs, ts, ms = [], [], []
    for i, nao in enumerate((256, 384, 512, 640, 768)):
        B, be, orbs = _packed_sequence(torch, ctx, nao, 40 + i, 10)
        x, t, m = controller.collect_samples(ctx, B, be, orbs, layout=DF_PACKED)
        xs.append(x), ts.append(t), ms.append(m)
        del B, be, orbs
    x, t, m = np.concatenate(xs), np.concatenate(ts), np.concatenate(ms)
    params, losses = controller.train(ctx, x, t, m, steps=4000, batch=512, lr=2e-3, seed=0)
    floor = controller.residual_floor(ctx, params, x, t, m, q=0.9)
    print(f"{x.shape[0]} samples, rms {controller.evaluate(ctx, params, x, t, m):.3f} decades, "
          f"floor {np.round(floor, 2).tolist()}")

    nao, n_iter = 1024, 20
    B, be, orbs = _packed_sequence(torch, ctx, nao, 7, n_iter)
    ctx.df_set_block_precision(None)
    ctx.ensure_workspace(4 * nao, nao, nao // 8)
    D = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    J, K = torch.empty_like(D), torch.empty_like(D)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_density(orbs[0], 2.0, D)
    costs = controller.build_costs(ctx, B, be, orbs[0], 2.0, D, J, K, en, eb, layout=DF_PACKED)
    print(f"uniform build ms at s = 1..8: {np.round(costs, 2).tolist()}")
    plain = adaptive.run_sequence(ctx, B, be, orbs, fp64_check=True, layout=DF_PACKED)
    ctl = controller.run_controlled(ctx, B, be, orbs, params, fp64_check=True, layout=DF_PACKED,
                                    s_refs=[r["slices"] for r in plain], floor=floor, cost=costs,
                                    min_gain=0.1, spot=1)
    ms_plain = sum(r["ms"] for r in plain)
    ms_ctl = sum(r["ms"] for r in ctl)
    for a, c in zip(plain, ctl):
        print(f"it {a['iteration']} plain s={a['slices']} {a['ms']:.1f} ms "
              f"err={a['k_maxabs_rel_fro']:.2e} | ctl work {c['work']}/{c['work_ref']} "
              f"{c['ms']:.1f} ms err={c['k_maxabs_rel_fro']:.2e} fb={c['fallback']} {c['mode']}")
    e_plain = max(r["k_maxabs_rel_fro"] for r in plain)
    e_ctl = max(r["k_maxabs_rel_fro"] for r in ctl)
    print(f"time: controller {ms_ctl:.1f} ms vs plain {ms_plain:.1f} ms "
          f"({ms_plain / ms_ctl:.3f}x); max K error {e_ctl:.2e} vs {e_plain:.2e}")
    ctx.close()
    assert any(c["mode"] == "controller" for c in ctl)
    assert ms_ctl < ms_plain
    assert e_ctl <= e_plain
