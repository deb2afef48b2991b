"""Oracle parity at the workload configurations the other GPU tests cover
only in part (one alignment pass of Algorithm 1 each):

* the 1000-particle case (L = 64, K = 10, shifts +-2, rings 1..30, SNR 0.1)
  in full, for the FP32, BF16 and FP16 contractions;
* every FP32 tile variant where the tuner uses it: the 4-wave resident
  variant at R4 = 12 (L = 96, rings 1..46) and the streamed variant at
  R4 = 12 and R4 = 16 (L = 128, rings 1..62);
* uneven stacks at full size: the two cheapest-to-check stacks of each box
  size of the 64-stack uneven distribution, aligned in one batched call
  (FP32 with the tuner's variants forced where they apply, and BF16), with
  32 sampled particles of each stack against the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth
from parity import agreement, check_align, check_pose, check_rescored_cc, pose_gap

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
TOL = {"fp32": 1e-5, "bf16": 2e-3, "fp16": 2e-3}


def log(msg):
    print(f"[gpu-configs] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def geom(sp, T=None):
    return oracle.Geometry(L=sp["L"], r_min=sp["r_min"], r_max=sp["r_max"], n_phi=256,
                           shift_max=sp["shift_max"] if T is None else T)


# ------------------------------------------------- 1000 particles, in full ---

@pytest.fixture(scope="module")
def small():
    w = synth.WORKLOADS["mra_small"]
    blobs = synth.make_blobs(w["K"], w["L"], seed=(w["seed"], 0), rho_max=w["rho_max"])
    refs = synth.render_refs(blobs).to(DEV)
    parts, _ = synth.make_particles(blobs, w["N"], w["shift_max"], w["snr"], seed=(w["seed"], 1), device=DEV)
    torch.cuda.synchronize()
    pn, rn = parts.cpu().numpy(), refs.cpu().numpy()
    g = geom(w)
    log(f"oracle on all {w['N']} particles")
    want = oracle.align(pn, rn, g)
    n_gap = 200
    gap = pose_gap(oracle.cc_table(pn[:n_gap], rn, g))
    qhat, _ = oracle.reference_polar(rn, g)
    return w, refs, parts, pn, want, gap, qhat, g


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_thousand_particles_in_full(ctx, small, precision):
    w, refs, parts, pn, want, gap, qhat, g = small
    log(f"{w['N']} particles, {precision}")
    ctx.load_refs(50, refs, r_min=w["r_min"], r_max=w["r_max"], shift_max=w["shift_max"], precision=precision)
    got = ctx.align(50, parts).to_numpy()
    err, frac = check_align(got, want, TOL[precision])
    agree = agreement(got, want)
    msg = f"  max rel CC err {err:.2e}, decided {frac:.3f}, equal parameters {agree.sum()}/{w['N']}"
    if precision == "fp32":
        assert agree.mean() >= 0.99, msg
    else:
        sub = {k: v[:len(gap)] for k, v in got.items()}
        wsub = {k: v[:len(gap)] for k, v in want.items()}
        n_pose = check_pose(sub, wsub, gap, TOL[precision], min_decided=len(gap) // 4)
        check_rescored_cc({k: v[:64] for k, v in got.items()}, pn[:64], qhat, g)
        assert agree.mean() >= 0.9, msg
        msg += f", decided by pose {n_pose}/{len(gap)}"
    log(msg)
    ctx.unload_refs(50)


# ------------------------------------------------------ FP32 tile variants ---

@pytest.mark.parametrize("L,r_max,variant", [(96, 46, 1), (96, 46, 2), (128, 62, 2)])
def test_fp32_variants_where_the_tuner_uses_them(ctx, L, r_max, variant):
    """R4 = ceil(rings / 4) = 12 and 16: the operand of the 8-wave resident
    variant no longer fits the registers, so the 4-wave resident (R4 <= 12)
    or the streamed variant runs."""
    log(f"fp32 variant {variant} at L={L} rings 1..{r_max}")
    K, T, N = 12, 2, 11
    blobs = synth.make_blobs(K, L, seed=(80 + variant, 0), rho_max=L / 2 - 4)
    refs = synth.render_refs(blobs).to(DEV)
    parts, _ = synth.make_particles(blobs, N, T, 0.1, seed=(80 + variant, 1), device=DEV)
    ctx.load_refs(51, refs, r_min=1, r_max=r_max, shift_max=T)
    ctx.set_tuning(51, corr_variant=variant)
    assert ctx.get_tuning(51)[0] == variant
    got = ctx.align(51, parts, with_cc2=True).to_numpy()
    g = oracle.Geometry(L=L, r_min=1, r_max=r_max, n_phi=256, shift_max=T)
    want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), g)
    err, frac = check_align(got, want, 1e-5)
    rel2 = np.abs(got["cc2"] - want["cc2"]) / np.abs(want["cc"])
    assert rel2.max() <= 1e-5
    log(f"  max rel CC err {err:.2e}, cc2 {rel2.max():.2e}, decided {frac:.3f}")
    ctx.unload_refs(51)


# ------------------------------------------- uneven stacks at full size ---

def _cheapest_stacks(per_L=2):
    specs = synth.uneven_stack_specs()
    cost = lambda sp: sp["K"] * (2 * sp["shift_max"] + 1) ** 2 * (sp["r_max"] - sp["r_min"] + 1)  # noqa: E731
    chosen = []
    for L in (64, 76, 96, 128):
        cands = sorted((i for i, sp in enumerate(specs) if sp["L"] == L), key=lambda i: cost(specs[i]))
        chosen += cands[:per_L]
    return [(i, specs[i]) for i in chosen]


@pytest.fixture(scope="module")
def uneven():
    data = []
    for i, sp in _cheapest_stacks():
        blobs = synth.make_blobs(sp["K"], sp["L"], seed=sp["seed"], rho_max=sp["rho_max"])
        refs = synth.render_refs(blobs).to(DEV)
        parts, _ = synth.make_particles(blobs, sp["N"], sp["shift_max"], sp["snr"], seed=(sp["seed"], 1),
                                        device=DEV)
        rng = np.random.default_rng(100 + i)
        idx = np.unique(np.concatenate([[0, sp["N"] - 1], rng.integers(0, sp["N"], 30)]))
        data.append((i, sp, refs, parts, idx))
    torch.cuda.synchronize()
    log(f"{len(data)} stacks, {sum(p.shape[0] for _, _, _, p, _ in data)} particles")
    want = []
    for i, sp, refs, parts, idx in data:
        sample = parts[torch.as_tensor(idx, device=DEV)].cpu().numpy()
        want.append((sample, oracle.align(sample, refs.cpu().numpy(), geom(sp))))
    return data, want


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_uneven_stacks_full_size_sampled_against_the_oracle(ctx, uneven, precision):
    from paper_2011_05755_amd import mra
    data, want = uneven
    base = 300 if precision == "fp32" else 400
    stacks = []
    for j, (i, sp, refs, parts, idx) in enumerate(data):
        ctx.load_refs(base + j, refs, r_min=sp["r_min"], r_max=sp["r_max"], shift_max=sp["shift_max"],
                      precision=precision)
        R4 = (sp["r_max"] - sp["r_min"] + 4) // 4
        if precision == "fp32" and 9 < R4 <= 12 and j % 2 == 0:
            ctx.set_tuning(base + j, corr_variant=1)      # the 4-wave resident form on half the L = 96 stacks
        stacks.append((base + j, parts, -1, mra.AlignResult.empty(parts.shape[0], DEV)))
    log(f"{precision}: one batched call over {len(stacks)} full-size stacks")
    ctx.align_batch(stacks)
    torch.cuda.synchronize()
    tol = TOL[precision]
    for (i, sp, refs, parts, idx), (sample, w), (_, _, _, out) in zip(data, want, stacks):
        got = {k: v[idx] for k, v in out.to_numpy().items()}
        err, frac = check_align(got, w, tol)
        if precision != "fp32":
            g = geom(sp)
            qhat, _ = oracle.reference_polar(refs.cpu().numpy(), g)
            check_rescored_cc(got, sample, qhat, g)
        log(f"  stack {i} (L={sp['L']} N={sp['N']} K={sp['K']} T={sp['shift_max']}): {len(idx)} sampled, "
            f"max rel CC err {err:.2e}, decided {frac:.2f}, equal {agreement(got, w).sum()}")
    for j in range(len(stacks)):
        ctx.unload_refs(base + j)
