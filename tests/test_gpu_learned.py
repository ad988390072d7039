"""Learned coarse correction of the FGMRES preconditioner: the library's
coarse restriction/prolongation, network forward, loss gradient and Adam
kernels against the FP64 oracle (oracle/learned.py), BF16 inference inside
the preconditioner, the fallback rule, and what the trained network gains
over the plain multi-level preconditioner."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu


def _rel(a, b):
    """Element-wise: largest entry difference over the largest reference entry."""
    a, b = np.ravel(a), np.ravel(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("case", [dict(dim=3, n_elem=4, m=2, p=2, periodic=True),
                                  dict(dim=2, n_elem=6, m=3, p=2, periodic=False, state="shear", mach=0.2)])
def test_coarse_restrict_prolong(case):
    import torch
    from oracle import learned as Ld
    say(f"[coarse] {case}")
    S, inp, ctx = make_pair(case)
    M = S.mesh
    F = ctx.coarse_size()
    assert F == Ld.n_features(M.dim)
    v = np.random.default_rng(11).standard_normal(M.n_glob)
    X = torch.empty(M.n_macros, F, dtype=torch.float32, device="cuda")
    ctx.coarse_restrict(to_dev(v), X)
    Xo = Ld.coarse_restrict(M, v)
    e = _rel(X.cpu().numpy(), Xo)
    say(f"[coarse] restrict rel err {e:.2e}")
    assert e < 1e-6
    Y = np.random.default_rng(12).standard_normal((M.n_macros, F)).astype(np.float32)
    z0 = np.random.default_rng(13).standard_normal(M.n_glob)
    z = to_dev(z0)
    ctx.coarse_prolong(torch.tensor(Y, device="cuda"), 0.5, z)
    zo = z0 + 0.5 * Ld.coarse_prolong(M, Y.astype(np.float64))
    e = _rel(z.cpu().numpy(), zo)
    say(f"[coarse] prolong rel err {e:.2e}")
    assert e < 1e-13


def _net_pair(ctx, hidden, batch, seed):
    import torch
    from oracle import learned as Ld
    from paper_2402_11361_amd.learned import CoarseCorrection
    cc = CoarseCorrection(ctx, hidden=hidden, max_batch=batch, seed=seed)
    rng = np.random.default_rng(seed + 100)
    F = cc.F
    P = Ld.init_params(F, hidden, F, rng)
    P["b1"] = 0.1 * rng.standard_normal(hidden)
    P["b2"] = 0.1 * rng.standard_normal(F)
    flat32 = Ld.flat(P).astype(np.float32)
    cc.params.copy_(torch.tensor(flat32, device="cuda"))
    P32 = Ld.unflat(flat32.astype(np.float64), F, hidden, F)
    return cc, P32


def test_mlp_forward_gradient_adam_against_oracle():
    import torch
    from oracle import learned as Ld
    say("[mlp] forward / gradient / Adam")
    S, inp, ctx = make_pair(dict(dim=3, n_elem=4, m=2, p=2, periodic=True))
    hidden, batch, N = 256, 96, 160
    cc, P = _net_pair(ctx, hidden, batch, seed=4)
    F = cc.F
    rng = np.random.default_rng(5)
    X = rng.standard_normal((N, F)).astype(np.float32)
    X[7] = 0.0  # a zero row maps to zero
    T = (0.3 * rng.standard_normal((N, F))).astype(np.float32)
    idx = rng.choice(N, batch, replace=False).astype(np.int32)
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    idd = torch.tensor(idx, device="cuda")
    Y = torch.empty(batch, F, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(cc.net, Xd, idd, batch, Y)
    Yo = Ld.forward(P, X[idx].astype(np.float64))
    e = _rel(Y.cpu().numpy(), Yo)
    say(f"[mlp] forward rel err {e:.2e}")
    assert e < 1e-5
    ctx.mlp_loss_grad(cc.net, Xd, Td, idd, batch, cc.loss)
    lo, Go = Ld.loss_and_grads(P, X[idx].astype(np.float64), T[idx].astype(np.float64))
    g = cc.grads.cpu().numpy().astype(np.float64)
    Gg = Ld.unflat(g, F, hidden, F)
    el = abs(float(cc.loss.item()) - lo) / lo
    say(f"[mlp] loss {lo:.6e} rel err {el:.2e}")
    assert el < 1e-5
    for k in ("W1", "b1", "W2", "b2"):
        e = _rel(Gg[k], Go[k])
        say(f"[mlp] grad {k} rel err {e:.2e}")
        assert e < 1e-5
    # one Adam step from zero moments with the GPU gradient
    Mo = {k: np.zeros_like(v) for k, v in P.items()}
    Vo = {k: np.zeros_like(v) for k, v in P.items()}
    Po = {k: v.copy() for k, v in P.items()}
    Ld.adam_step(Po, Gg, Mo, Vo, 1, lr=1e-3)
    ctx.mlp_adam(cc.net, 1e-3, 0.9, 0.999, 1e-8, 1)
    Pg = Ld.unflat(cc.params.cpu().numpy().astype(np.float64), F, hidden, F)
    for k in Po:
        e = np.abs(Pg[k] - Po[k]).max()
        assert e < 1e-6, (k, e)


def test_bf16_inference_in_preconditioner():
    import torch
    from oracle import learned as Ld
    say("[bf16] learned stage inside the preconditioner")
    S, inp, ctx = make_pair(dict(dim=3, n_elem=4, m=2, p=2, periodic=True))
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    cc, P = _net_pair(ctx, 256, 64, seed=8)
    cc.bind()
    v = np.random.default_rng(9).standard_normal(ctx.n_glob)
    zp = torch.empty(ctx.n_glob, dtype=torch.float64, device="cuda")
    zl = torch.empty_like(zp)
    ctx.precond_apply(to_dev(v), zp, 5)
    ctx.precond_apply(to_dev(v), zl, 5, use_learned=True)
    got = (zl - zp).cpu().numpy()
    M = S.mesh
    ref = Ld.coarse_prolong(M, Ld.forward(P, Ld.coarse_restrict(M, v)))
    e = _rel(got, ref)
    say(f"[bf16] correction rel err vs FP64 oracle {e:.2e}")
    # BF16 weights (8-bit significand, relative rounding 2^-9) with FP32 sums
    assert e < 2e-2
    assert e > 1e-6  # the BF16 copy is what ran


CASE_TRAIN = dict(dim=3, n_elem=8, m=2, p=2, periodic=True, mach=0.1, Re=1600.0, noise=1e-4)


def _condensed(seed):
    import torch
    S, inp, ctx = make_pair(dict(CASE_TRAIN, seed=seed))
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    return ctx, bhat


@pytest.fixture(scope="module")
def trained():
    """A network trained on pairs harvested from two seeded states."""
    import torch
    from paper_2402_11361_amd.learned import CoarseCorrection
    say("[train] harvesting")
    cc = None
    for seed in (0, 1):
        ctx, bhat = _condensed(seed)
        if cc is None:
            cc = CoarseCorrection(ctx, hidden=256, max_batch=512, seed=0)
        else:
            cc.ctx = ctx
        k = cc.harvest(bhat, n_vectors=30)
        say(f"[train] seed {seed}: {k} vectors, {cc.n_pairs()} pairs")
    X = torch.cat(cc.X)
    T = torch.cat(cc.T)
    loss0 = cc.eval_loss(X, T)
    hist = cc.train(epochs=150, lr=1e-3, batch=512)
    loss1 = cc.eval_loss(X, T)
    say(f"[train] loss {loss0:.4e} -> {loss1:.4e} (epochs: first {hist[0]:.4e} last {hist[-1]:.4e})")
    return cc, loss0, loss1


def test_training_reduces_loss(trained):
    cc, loss0, loss1 = trained
    assert loss1 < 0.7 * loss0


def _held_out(cc):
    """A fresh context on a held-out state, with its plain solve."""
    import torch
    ctx, bhat = _condensed(5)
    xp = torch.zeros_like(bhat)
    ip = ctx.fgmres_solve(bhat, xp, rtol=1e-10, restart=30, inner_its=5)
    assert ip["converged"]
    return ctx, bhat, xp, ip


@pytest.mark.xfail(reason="no gain measured: the trained correction is local per macro while the error the plain "
                          "multi-level preconditioner leaves is global; held-out solves need more outer iterations "
                          "with the learned stage than without it", strict=False)
def test_learned_gain_without_fallback(trained):
    """What the trained network gains on its own: the held-out solve with the
    learned stage kept for the whole solve (no fallback) against the plain
    multi-level preconditioner."""
    import torch
    cc, _, _ = trained
    ctx, bhat, xp, ip = _held_out(cc)
    cc.ctx = ctx
    cc.bind()
    xl = torch.zeros_like(bhat)
    il = ctx.fgmres_solve(bhat, xl, rtol=1e-10, restart=30, inner_its=5, use_learned=True, no_fallback=True)
    say(f"[gain] plain: {ip['outer_its']} outer its, {ip['ms']:.1f} ms;  learned (no fallback): "
        f"{il['outer_its']} outer its, {il['ms']:.1f} ms")
    assert il["converged"] and il["fallbacks"] == 0
    assert float((xl - xp).norm() / xp.norm()) < 1e-6
    assert il["outer_its"] < ip["outer_its"]


def test_learned_stage_judged_by_plain_on_fresh_context(trained):
    """With fallback on, a solve is never worse than the plain judge allows and
    keeps the plain solution; a deliberately broken (scaled) network on a fresh
    context, with no plain solve before it, is switched off by its own solve's
    plain steps."""
    import torch
    cc, _, _ = trained
    ctx, bhat, xp, ip = _held_out(cc)
    cc.ctx = ctx
    cc.bind()
    xl = torch.zeros_like(bhat)
    il = ctx.fgmres_solve(bhat, xl, rtol=1e-10, restart=30, inner_its=5, use_learned=True)
    say(f"[judge] plain {ip['outer_its']} its; learned with fallback {il['outer_its']} its, "
        f"fallbacks {il['fallbacks']}")
    assert il["converged"] and float((xl - xp).norm() / xp.norm()) < 1e-6
    # fresh context: no plain history at all before the learned solve
    ctx2, bhat2 = _condensed(5)
    cc.ctx = ctx2
    saved = cc.params.clone()
    cc.params.mul_(40.0)
    cc.bind()
    cc.params.copy_(saved)
    xb = torch.zeros_like(bhat2)
    ib = ctx2.fgmres_solve(bhat2, xb, rtol=1e-10, restart=30, inner_its=5, use_learned=True)
    say(f"[fallback] fresh context, scaled network: {ib['outer_its']} outer its, fallbacks {ib['fallbacks']}")
    assert ib["converged"] and ib["fallbacks"] == 1
    assert float((xb - xp).norm() / xp.norm()) < 1e-6
    # the same on the graph-captured path
    xg = torch.zeros_like(bhat2)
    cc.params.mul_(40.0)
    cc.bind()
    cc.params.copy_(saved)
    ig = ctx2.fgmres_solve(bhat2, xg, rtol=1e-10, restart=30, inner_its=5, use_learned=True, graph_steps=10)
    say(f"[fallback] graph steps, scaled network: {ig['outer_its']} outer its, fallbacks {ig['fallbacks']}")
    assert ig["converged"] and ig["fallbacks"] == 1
    assert float((xg - xp).norm() / xp.norm()) < 1e-6


def test_graphs_follow_rebound_network_width(trained):
    """Captured FGMRES steps are rebuilt when a network of another hidden
    width is bound: graph-mode solves match host-controlled solves with each
    width in turn (learned stage kept, no fallback)."""
    import torch
    from paper_2402_11361_amd.learned import CoarseCorrection
    cc, _, _ = trained
    ctx, bhat = _condensed(5)
    small = CoarseCorrection(ctx, hidden=64, max_batch=64, seed=3)
    for net in (cc, small, cc):
        net.ctx = ctx
        net.bind()
        xh = torch.zeros_like(bhat)
        ih = ctx.fgmres_solve(bhat, xh, rtol=1e-10, restart=30, inner_its=5, use_learned=True, no_fallback=True)
        xg = torch.zeros_like(bhat)
        ig = ctx.fgmres_solve(bhat, xg, rtol=1e-10, restart=30, inner_its=5, use_learned=True, no_fallback=True,
                              graph_steps=10)
        say(f"[graph] hidden {net.hidden}: host {ih['outer_its']} its, graph {ig['outer_its']} its")
        assert ih["converged"] and ig["converged"]
        assert abs(ih["outer_its"] - ig["outer_its"]) <= 1
        assert float((xg - xh).norm() / xh.norm()) < 1e-8


@pytest.mark.parametrize("case", [dict(dim=3, n_elem=4, m=2, p=2, periodic=True),
                                  dict(dim=2, n_elem=6, m=3, p=2, periodic=False, state="shear", mach=0.2)])
def test_neighbour_features_and_inference_against_oracle(case):
    """hdg_coarse_neighbours against the oracle's neighbour features, and the
    learned stage of a network fed by them (n_in = (1 + 2d) F) inside the
    preconditioner against the FP64 oracle."""
    import torch
    from oracle import learned as Ld
    from paper_2402_11361_amd.learned import CoarseCorrection
    say(f"[neighbours] {case}")
    S, inp, ctx = make_pair(case)
    M = S.mesh
    F = ctx.coarse_size()
    v = np.random.default_rng(21).standard_normal(M.n_glob)
    X = torch.empty(M.n_macros, F, dtype=torch.float32, device="cuda")
    ctx.coarse_restrict(to_dev(v), X)
    Xe = torch.empty(M.n_macros, (1 + 2 * M.dim) * F, dtype=torch.float32, device="cuda")
    ctx.coarse_neighbours(X, Xe)
    # the gather is a copy: exact against the oracle's gather of the GPU's X
    assert np.array_equal(Xe.cpu().numpy(), Ld.neighbour_features(M, X.cpu().numpy().astype(np.float64)))
    Xo = Ld.neighbour_features(M, Ld.coarse_restrict(M, v))
    e = _rel(Xe.cpu().numpy(), Xo)
    say(f"[neighbours] features rel err {e:.2e}")
    assert e < 1e-6
    d = {k: (to_dev(w) if isinstance(w, np.ndarray) else w) for k, w in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    hidden = 128
    cc = CoarseCorrection(ctx, hidden=hidden, max_batch=64, seed=3, neighbours=True)
    rng = np.random.default_rng(33)
    n_in = cc.n_in
    P = Ld.init_params(n_in, hidden, F, rng)
    P["b1"] = 0.1 * rng.standard_normal(hidden)
    P["b2"] = 0.1 * rng.standard_normal(F)
    flat32 = Ld.flat(P).astype(np.float32)
    cc.params.copy_(torch.tensor(flat32, device="cuda"))
    P32 = Ld.unflat(flat32.astype(np.float64), n_in, hidden, F)
    cc.bind()
    zp = torch.empty(ctx.n_glob, dtype=torch.float64, device="cuda")
    zl = torch.empty_like(zp)
    ctx.precond_apply(to_dev(v), zp, 5)
    ctx.precond_apply(to_dev(v), zl, 5, use_learned=True)
    got = (zl - zp).cpu().numpy()
    ref = Ld.coarse_prolong(M, Ld.forward(P32, Xo))
    e = _rel(got, ref)
    say(f"[neighbours] correction rel err vs FP64 oracle {e:.2e}")
    assert 1e-6 < e < 2e-2  # BF16 weights, FP32 sums
    ctx.close()


@pytest.fixture(scope="module")
def trained_neighbours():
    """The trained network of the other fixture's recipe, fed the coarse
    coefficients of the face neighbours too."""
    import torch
    from paper_2402_11361_amd.learned import CoarseCorrection
    cc = None
    for seed in (0, 1):
        ctx, bhat = _condensed(seed)
        if cc is None:
            cc = CoarseCorrection(ctx, hidden=256, max_batch=512, seed=0, neighbours=True)
        else:
            cc.ctx = ctx
        cc.harvest(bhat, n_vectors=30)
    X = torch.cat(cc.X)
    T = torch.cat(cc.T)
    loss0 = cc.eval_loss(X, T)
    cc.train(epochs=150, lr=1e-3, batch=512)
    loss1 = cc.eval_loss(X, T)
    say(f"[train neighbours] {cc.n_pairs()} pairs, loss {loss0:.4e} -> {loss1:.4e}")
    return cc, loss0, loss1


def test_training_with_neighbours_reduces_loss(trained_neighbours, trained):
    cc, loss0, loss1 = trained_neighbours
    _, p0, p1 = trained
    say(f"[train neighbours] final loss {loss1:.4e} (own macro only: {p1:.4e})")
    assert loss1 < 0.7 * loss0


@pytest.mark.xfail(reason="no gain measured: the held-out solve with the neighbour-fed network kept for the whole "
                          "solve needs as many or more outer iterations than the plain preconditioner", strict=False)
def test_learned_gain_with_neighbours_without_fallback(trained_neighbours):
    """The held-out solve with the neighbour-fed network kept for the whole
    solve against the plain multi-level preconditioner."""
    import torch
    cc, _, _ = trained_neighbours
    ctx, bhat, xp, ip = _held_out(cc)
    cc.ctx = ctx
    cc.bind()
    xl = torch.zeros_like(bhat)
    il = ctx.fgmres_solve(bhat, xl, rtol=1e-10, restart=30, inner_its=5, use_learned=True, no_fallback=True)
    say(f"[gain neighbours] plain: {ip['outer_its']} outer its, {ip['ms']:.1f} ms;  learned (no fallback): "
        f"{il['outer_its']} outer its, {il['ms']:.1f} ms")
    assert il["converged"] and il["fallbacks"] == 0
    assert float((xl - xp).norm() / xp.norm()) < 1e-6
    assert il["outer_its"] < ip["outer_its"]
