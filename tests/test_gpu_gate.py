"""The learned gate on the GPU against its CPU reference and the oracle.

Inference: logits of the BF16 MFMA kernel vs the CPU forward pass with the
same BF16 roundings (FP64 accumulation) within 1e-3.  Harvest: features and
the WENO weight deviation vs the CPU definitions.  Gated step: the GPU step
with the gate on vs the oracle's gated step, whose flags come from the CPU
forward pass (the threshold is placed in a gap of the CPU logits so the
decision is unambiguous).  Training: GPU gradients vs FP64 CPU gradients,
and the loss falls.
"""
import numpy as np
import pytest

import icgen
import oracle
from oracle import gate as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def random_params(nf, seed):
    p = cg.init_params(nf, seed=seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["b2"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["b3"] = np.array([0.05], np.float32)
    return p


def vec(hog, p):
    return hog.pack_params(p["W1"], p["b1"], p["W2"], p["b2"], p["w3"], p["b3"])


@pytest.mark.parametrize("ndim", [2, 3])
def test_gate_logits_match_cpu(hog, ndim):
    n = (20, 18, 16) if ndim == 3 else (40, 36, 1)
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=3, amp=0.3)
    nf = (ndim + 2) * (4 * ndim + 1)
    p = random_params(nf, seed=ndim)
    g = hog.Grid.from_problem(pb, 4)
    g.set_gate(vec(hog, p), theta=0.5)
    logits, flags = g.gate_eval()
    ref, _ = cg.forward(p, cg.features(pb.U, ndim, pb.bc))
    ref = ref.reshape(logits.shape)
    np.testing.assert_allclose(logits, ref, rtol=0, atol=1e-3 * max(1.0, np.abs(ref).max()))
    sure = np.abs(ref) > 1e-2
    np.testing.assert_array_equal(flags[sure], (ref[sure] >= 0).astype(np.uint8))


@pytest.mark.parametrize("ndim,order", [(2, 3), (3, 4)])
def test_harvest_matches_definitions(hog, ndim, order):
    pb = icgen.multiblast(n=14, seed=3) if ndim == 3 else icgen.sod(n=30, axis=1, ndim=2, ntrans=26)
    g = hog.Grid.from_problem(pb, order)
    N = pb.U[0].size
    zones = np.arange(0, N, 3)
    F, dev = g.harvest(zones)
    Fc = cg.features(pb.U, ndim, pb.bc)[zones]
    np.testing.assert_allclose(F.cpu().numpy(), Fc, rtol=0, atol=1e-6)
    dc = oracle.zone_maxdev(oracle.cfg_from_problem(pb, order), pb.U).reshape(-1)[zones]
    np.testing.assert_allclose(dev.cpu().numpy(), dc, rtol=1e-5, atol=1e-7)
    assert (dc > 0.25).any() and (dc <= 0.25).any()


@pytest.mark.parametrize("ndim,order", [(2, 3), (3, 4)])
def test_gated_step_matches_oracle(hog, ndim, order):
    n = (16, 14, 12) if ndim == 3 else (40, 36, 1)
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=8, amp=0.3)
    nf = (ndim + 2) * (4 * ndim + 1)
    p = random_params(nf, seed=10 + ndim)
    ref, _ = cg.forward(p, cg.features(pb.U, ndim, pb.bc))
    # threshold in the widest gap of the CPU logits near their median
    srt = np.sort(ref)
    mid = len(srt) // 2
    lo, hi = max(1, mid - len(srt) // 4), min(len(srt) - 1, mid + len(srt) // 4)
    k = lo + int(np.argmax(np.diff(srt[lo - 1:hi])))
    thr = 0.5 * (srt[k - 1] + srt[k])
    assert srt[k] - srt[k - 1] > 2e-3
    flags = (ref >= thr).astype(np.uint8).reshape(pb.U[0].shape)
    assert 0 < flags.sum() < flags.size
    theta = 1.0 / (1.0 + np.exp(-thr))
    g = hog.Grid.from_problem(pb, order)
    g.set_gate(vec(hog, p), theta=theta)
    _, fg = g.gate_eval()
    np.testing.assert_array_equal(fg, flags)
    c = oracle.cfg_from_problem(pb, order)
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    U = g.get_state()
    Uo, _ = oracle.step_gated(c, pb.U, dt, flags)
    assert np.abs(U - Uo).sum() / np.abs(Uo).sum() <= 1e-12
    # and the gate did change the solution
    assert np.abs(Uo - oracle.step(c, pb.U, dt)).max() > 1e-10


@pytest.mark.parametrize("ndim,order", [(2, 4), (3, 4), (3, 3)])
def test_fixed_gate_flags_step_matches_oracle(hog, ndim, order):
    """Caller-set flags (a seeded random selection, as in the gate ablations)
    give the oracle's gated step for the same flags."""
    n = (16, 14, 12) if ndim == 3 else (40, 36, 1)
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=20 + order, amp=0.3)
    flags = (np.random.default_rng(ndim + order).uniform(size=pb.U[0].shape) < 0.4).astype(np.uint8)
    c = oracle.cfg_from_problem(pb, order)
    dt, _ = oracle.cfl_dt(c, pb.U)
    g = hog.Grid.from_problem(pb, order)
    g.set_gate_flags(flags)
    g.step(dt)
    Uo, _ = oracle.step_gated(c, pb.U, dt, flags)
    assert np.abs(g.get_state() - Uo).sum() / np.abs(Uo).sum() <= 1e-12
    with pytest.raises(hog.HogError):
        g.gate_eval()                                   # no network, fixed flags
    bad = flags.copy()
    bad.flat[3] = 2
    with pytest.raises(hog.HogError):
        g.set_gate_flags(bad)
    g.set_gate_flags(None)                              # back to no gate: the plain step
    g.set_state(pb.U)
    g.step(dt)
    assert np.abs(g.get_state() - oracle.step(c, pb.U, dt)).sum() / np.abs(Uo).sum() <= 1e-12


def test_mlp_gradients_match_cpu(hog):
    rng = np.random.default_rng(1)
    nf, B = 65, 256
    X = rng.normal(size=(B, nf)).astype(np.float32)
    y = (rng.uniform(size=B) < 0.4).astype(np.float32)
    w = np.where(y > 0, 1.25, 0.8).astype(np.float32)
    p = random_params(nf, seed=4)
    m = hog.Mlp(nf, batch_max=512)
    m.set_params(vec(hog, p))
    loss, gvec = m.grads(X, y, w)
    Lc, gc = cg.loss_and_grads(p, X.astype(np.float64), y, w)
    assert abs(loss - Lc) <= 1e-5 * abs(Lc)
    G = hog.unpack_params(gvec, nf)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        ref = gc[k].reshape(G[k].shape)
        err = np.linalg.norm(G[k] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err <= 1e-3, (k, err)


def test_mlp_training_separates_harvested_labels(hog):
    import torch
    samples, labels = [], []
    for pb in (icgen.vortex3d_perturbed(n=24, seed=2), icgen.multiblast(n=24, seed=3)):
        g = hog.Grid.from_problem(pb, 4)
        for _ in range(3):
            F, dev = g.harvest(np.arange(pb.U[0].size))
            samples.append(F)
            labels.append((dev <= 0.25).float())
            g.advance(2)
    X = torch.cat(samples)
    y = torch.cat(labels)
    frac = float(y.mean())
    w = torch.where(y > 0, 0.5 / frac, 0.5 / (1 - frac)).float()
    m = hog.Mlp(65, batch_max=4096)
    m.set_params(vec(hog, random_params(65, seed=0)))
    gen = torch.Generator(device="cpu").manual_seed(0)
    first = None
    for it in range(300):
        idx = torch.randint(0, X.shape[0], (4096,), generator=gen).cuda()
        loss = m.step(X[idx].contiguous(), y[idx].contiguous(), w[idx].contiguous(), lr=3e-3)
        if first is None:
            first = loss
    logits = m.predict(X)
    acc = float(((logits >= 0).float() == y).float().mean())
    print(f"gate training: smooth fraction {frac:.3f}, loss {first:.3f} -> {loss:.3f}, accuracy {acc:.4f}", flush=True)
    assert loss < 0.5 * first and acc > 0.9


GATE_FILE = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "paper_2211_13295_amd",
                                       "gate_o4_3d.npz")


def _run(hog, pb, steps, precision, gate=None):
    g = hog.Grid.from_problem(pb, 4, precision=precision)
    frac = []
    if gate is not None:
        g.set_gate(gate[0], theta=gate[1])
    for _ in range(steps):
        if gate is not None:
            frac.append(float(g.gate_eval()[1].mean()))
        g.advance(1)
    out = (g.get_state(), g.stats()["t"], float(np.mean(frac)) if frac else 0.0)
    g.close()
    return out


def test_trained_gate_gain_four_quadrant(hog):
    """What the network's selection gains on the headline workload, scaled
    down (four-quadrant Riemann problem, 64^3, fourth order, 20 steps, mixed
    path): a large share of the zones runs on the linear weights, and the
    state stays close to the FP64 path -- much closer than with the same share
    of zones chosen at random each step, or with linear weights everywhere."""
    z = np.load(GATE_FILE)
    gate = (z["params"], float(z["theta"]))
    pb = icgen.four_quadrant(n=64, seed=5)
    steps = 20
    ref, _, _ = _run(hog, pb, steps, "fp64")
    Ug, _, frac = _run(hog, pb, steps, "mixed", gate)
    rng = np.random.default_rng(9)
    g = hog.Grid.from_problem(pb, 4, precision="mixed")
    for _ in range(steps):
        g.set_gate_flags((rng.uniform(size=pb.U[0].shape) < frac).astype(np.uint8))
        g.advance(1)
    Ur = g.get_state()
    g.set_gate_flags(np.ones(pb.U[0].shape, np.uint8))
    g.set_state(pb.U)
    try:
        g.advance(steps)
        Ul = g.get_state()
    except hog.HogError:                 # linear weights at the discontinuities: a non-physical state
        Ul = np.full_like(ref, np.inf)
    g.close()
    Um, _, _ = _run(hog, pb, steps, "mixed")
    rel = {k: float(np.abs(U - ref).sum() / np.abs(ref).sum()) for k, U in
           (("gate", Ug), ("random", Ur), ("linear", Ul), ("mixed", Um))}
    print(f"gate gain, four-quadrant 64^3: {100 * frac:.1f}% of zones on linear weights; rel L1 vs FP64 {rel}",
          flush=True)
    assert frac > 0.3
    assert rel["gate"] <= 1e-3
    assert rel["random"] >= 5.0 * rel["gate"] and rel["linear"] >= 5.0 * rel["gate"]


def test_trained_gate_gain_smooth(hog):
    """What the trained gate buys on smooth flow with a known solution (the
    isentropic vortex extruded along z, 40^3, fourth order, 10 steps): the
    share of zones whose WENO applications run with the linear weights (no
    smoothness indicators, no epsilon division), at the density L1 error
    against the exact translated vortex of the ungated mixed path."""
    z = np.load(GATE_FILE)
    gate = (z["params"], float(z["theta"]))
    n, steps = 40, 10
    pb = icgen.vortex3d_perturbed(n=n, seed=2, amp=0.0)
    err, frac = {}, 0.0
    for mode in ("fp64", "mixed", "gated"):
        U, t, f = _run(hog, pb, steps, "fp64" if mode == "fp64" else "mixed", gate if mode == "gated" else None)
        err[mode] = float(np.abs(U[0] - icgen.vortex_exact_density(n, t)[None]).mean())
        frac = f if mode == "gated" else frac
    print(f"gate gain, smooth vortex: {100 * frac:.1f}% of zones on linear weights; density L1 error vs exact "
          f"{err['gated']:.4e} gated, {err['mixed']:.4e} mixed, {err['fp64']:.4e} FP64", flush=True)
    assert frac > 0.005
    assert err["gated"] <= 1.02 * err["mixed"]


def test_trained_gate_keeps_the_vortex_order_3d(hog):
    """The mixed path with the trained gate keeps the design order on the
    isentropic vortex extruded along z (fourth order, 32^3 -> 64^3 on
    [0,10]^3, to t = 1): the density L1 error against the exact translated
    vortex falls at least as fast as order 3.75, like the ungated mixed path's
    floor."""
    z = np.load(GATE_FILE)
    gate = (z["params"], float(z["theta"]))
    errs, fracs = [], []
    for n in (32, 64):
        pb = icgen.vortex3d_perturbed(n=n, seed=2, amp=0.0)
        g = hog.Grid.from_problem(pb, 4, precision="mixed")
        g.set_gate(gate[0], theta=gate[1])
        fracs.append(float(g.gate_eval()[1].mean()))
        t = g.advance(100000, t_end=1.0)
        ex = icgen.vortex_exact_density(n, t)
        errs.append(float(np.abs(g.get_state()[0] - ex[None]).mean()))
        g.close()
    rate = np.log2(errs[0] / errs[1])
    print(f"mixed + trained gate, 3D vortex: errors {errs}, order {rate:.2f}, gated fractions {fracs}", flush=True)
    assert rate >= 3.75


def test_trained_gate_gain_shocks(hog):
    """The same on the multi-blast (shocks, 40^3, 8 steps): most of the
    quiescent ambient runs on linear weights, full WENO stays in the blast
    zones, and the state stays within the mixed path's shock bound of the FP64
    path (relative L1)."""
    z = np.load(GATE_FILE)
    gate = (z["params"], float(z["theta"]))
    pb = icgen.multiblast(n=40, seed=3)
    ref, _, _ = _run(hog, pb, 8, "fp64")
    Ug, _, frac = _run(hog, pb, 8, "mixed", gate)
    Um, _, _ = _run(hog, pb, 8, "mixed")
    rel_g = np.abs(Ug - ref).sum() / np.abs(ref).sum()
    rel_m = np.abs(Um - ref).sum() / np.abs(ref).sum()
    print(f"gate gain, multi-blast: {100 * frac:.1f}% of zones on linear weights; rel L1 vs FP64 "
          f"{rel_g:.3e} gated, {rel_m:.3e} mixed", flush=True)
    assert frac > 0.5
    assert rel_g <= 1e-3
