"""Initial-guess network: the matrix-core kernels (BF16 and FP32 operands)
against the FP64 oracle network, and the learned guess inside the Krylov
solve of the cylinder workload (iterations saved, results unchanged)."""
import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import network as N
from oracle import geometry as OG
from oracle import ns as ONS
from gpu_util import DEV, to_dev, seeded_state, rel

pytestmark = pytest.mark.gpu

# FP32 operands: rounding of FP32 products through a few layers.  BF16
# operands: each product rounds both operands to 8 significant bits
# (relative 2^-9 each); the errors of independent roundings add in
# quadrature over a K-term sum, so a layer's relative error stays near
# 2^-9 (measured: forward 3.5e-3 and 5.5e-3, gradients at most 4.7e-3 and
# 7.3e-3 for widths 16 and 128), below the 2e-2 bound asked of the BF16 path.
TOL_F32_FWD, TOL_F32_GRAD = 1e-5, 1e-4
TOL_BF16_FWD, TOL_BF16_GRAD = 2e-2, 2e-2


def _segments(lengths):
    seg0, segl, pos, start = [], [], [], 0
    for L in lengths:
        for q in range(L):
            seg0.append(start)
            segl.append(L)
            pos.append(q)
        start += L
    return np.array([seg0, segl, pos], dtype=np.int32)


def _dev32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def _case(sizes, lengths, B, seed):
    rng = np.random.default_rng(seed)
    P = sum(lengths)
    X = rng.standard_normal((B, P, sizes[0]))
    T = rng.standard_normal((B, P))
    params = N.init_params(sizes, seed=seed + 1)
    # non-zero biases so that the bias paths are exercised
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    # round the oracle's inputs to FP32 so both sides see the same numbers
    X = X.astype(np.float32).astype(np.float64)
    T = T.astype(np.float32).astype(np.float64)
    flat = N.flatten(params).astype(np.float32)
    params = N.unflatten(flat.astype(np.float64), sizes)
    return X, T, params, flat


def _oracle(params, X, T, lengths):
    ys, grads, start = [], None, 0
    B, P = X.shape[:2]
    loss = 0.0
    for L in lengths:
        sl = slice(start, start + L)
        y, _ = N.forward(params, X[:, sl])
        ys.append(y[..., 0])
        l, g = N.loss_and_grads(params, X[:, sl], T[:, sl])
        w = (B * L) / (B * P)          # the batch loss is the mean over all B*P outputs
        loss += w * l
        gf = N.flatten([(gw * w, gb * w) for gw, gb in g])
        grads = gf if grads is None else grads + gf
        start += L
    return np.concatenate(ys, 1), loss, grads


SIZES = {"small": [10, 16, 16, 1], "paper": [10, 128, 128, 128, 1]}
LENGTHS = [37, 50, 3, 1, 70]


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("arch", list(SIZES))
def test_forward_and_gradients_match_oracle(arch, bf16):
    sizes = SIZES[arch]
    X, T, params, flat = _case(sizes, LENGTHS, B=3, seed=7)
    net = iim.Network(in_channels=sizes[0], width=sizes[1], layers=len(sizes) - 1, bf16=bf16)
    net.set(flat)
    seq = torch.as_tensor(_segments(LENGTHS), device=DEV)
    x, t = _dev32(X), _dev32(T)
    y = torch.zeros((X.shape[0], X.shape[1]), dtype=torch.float32, device=DEV)
    net.forward(x, seq, y)
    loss = net.grad_mse(x, seq, t)
    torch.cuda.synchronize()
    g = net.get(1).astype(np.float64)
    y_ref, loss_ref, g_ref = _oracle(params, X, T, LENGTHS)
    ey = rel(y.cpu().numpy(), y_ref)
    tf, tg = (TOL_BF16_FWD, TOL_BF16_GRAD) if bf16 else (TOL_F32_FWD, TOL_F32_GRAD)
    # every layer's weight and bias gradient
    off, eg = 0, []
    for cin, cout in zip(sizes[:-1], sizes[1:]):
        for n in (N.TAPS * cin * cout, cout):
            eg.append(rel(g[off:off + n], g_ref[off:off + n]))
            off += n
    print(arch, "bf16" if bf16 else "fp32", "forward", ey, "loss", abs(loss - loss_ref) / loss_ref, "gradients", eg)
    assert ey < tf, ey
    assert abs(loss - loss_ref) / loss_ref < tf, (loss, loss_ref)
    assert max(eg) < tg, eg


def test_adam_step_matches_oracle():
    sizes = SIZES["small"]
    X, T, params, flat = _case(sizes, [40, 24], B=2, seed=3)
    net = iim.Network(in_channels=sizes[0], width=sizes[1], layers=len(sizes) - 1, bf16=False)
    net.set(flat)
    seq = torch.as_tensor(_segments([40, 24]), device=DEV)
    x, t = _dev32(X), _dev32(T)
    p = flat.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        net.grad_mse(x, seq, t)
        g = net.get(1).astype(np.float64)
        net.adam_step(1e-2)
        p, m, v = N.adam_step(p, g, m, v, step, lr=1e-2)
        got = net.get(0).astype(np.float64)
        # the update itself (lr-sized) must agree to FP32 rounding
        assert np.max(np.abs(got - p)) < 1e-5, (step, np.max(np.abs(got - p)))
        p = got


def test_training_across_runs_and_validation_loss():
    """One network trained on the records of two runs of different viscosity
    and body position (iim_warm_start_train_multi) lowers the loss on both;
    the validation loss (iim_warm_start_loss) does not depend on how the
    records are batched and counts every record with three predecessors."""
    base = wl.cylinder_small()
    runs = []
    for re, dx in ((50.0, 0.0), (150.0, 0.3 * base.grid.h)):
        w = wl.cylinder(nx=base.grid.nx, ny=base.grid.ny, h=base.grid.h, points=128, dt=base.dt,
                        center=(1.5 + dx, 0.1 * dx), nu=1.0 / re)
        ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
        ctx.record_solves(200)
        om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device=DEV)
        ctx.rk3_steps(om, np.zeros(ctx.n_circ), w.dt, 40)
        runs.append(ctx)
    torch.cuda.synchronize()
    net = iim.Network(bf16=True, seed=0)
    before = [c.warm_start_loss(net)[0] for c in runs]
    for c in runs:
        l1, n1 = c.warm_start_loss(net, batch=1)
        l64, n64 = c.warm_start_loss(net, batch=64)
        assert n1 == n64 == 40 * 3 - 3
        assert abs(l1 - l64) < 1e-5 * l64, (l1, l64)
    losses = iim.warm_start_train_multi(runs, net, iters=300, batch=32, lr=1e-3, seed=4)
    assert np.all(np.isfinite(losses))
    after = [c.warm_start_loss(net)[0] for c in runs]
    print("validation losses before", before, "after", after)
    assert all(a < 0.7 * b for a, b in zip(after, before)), (before, after)
    for c in runs:
        c.close()


def test_sequences_cover_affected_points():
    w = wl.cylinder_small()
    ctx = iim.Context(w.grid, w.bodies)
    perm, seq, geo = ctx.warm_start_sequences()
    na = ctx.info["n_affected"]
    assert sorted(perm.tolist()) == list(range(na))
    a_int = ctx.geometry()["a_int"]
    assert np.array_equal(geo[:, 0], a_int[perm, 2].astype(np.float32))
    assert np.all((seq[2] >= 0) & (seq[2] < seq[1]))


def _run(ctx, omega0, G0, dt, steps):
    om = to_dev(omega0)
    ctx.reset_history()
    G = np.array(G0, dtype=np.float64)
    iters, res0 = [], []
    for _ in range(steps):
        G, st = ctx.rk3_steps(om, G, dt, 1)
        iters += st["iters"]
        res0 += st["res0"]
    torch.cuda.synchronize()
    return om.cpu().numpy(), G, np.array(iters), np.array(res0)


def _state(w, geo, seed):
    """Seed 0: the impulsive start from rest; otherwise mild domain-scale
    vortices added to it (the training runs)."""
    if seed == 0:
        return np.zeros((w.grid.ny, w.grid.nx)), np.zeros(geo.nbc)
    return np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, seed, count=8), 0.0), np.zeros(geo.nbc)


def test_learned_guess_in_the_krylov_solve():
    """Trains the network on recorded solves of perturbed runs, then solves
    the held-out impulsive start to 1e-10 with each initial guess.  Asserted:
    the network lowers the initial residual below the extrapolated guess it
    corrects; the extrapolated guess takes fewer Krylov iterations than the
    previous-stage guess; the network guess is not worse than the
    previous-stage guess in iterations (it does not beat the extrapolation:
    the iterations follow the error in the slowly converging directions,
    which the network does not reduce); the results do not depend on the
    guess."""
    w = wl.cylinder_small()
    geo = OG.Geometry(w.grid, w.bodies)
    rec = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    rec.record_solves(4000)
    for seed in range(1, 9):
        om, G = _state(w, geo, seed)
        _run(rec, om, G, w.dt, 60)
    assert rec.warm_start_stats()["recorded"] == 8 * 60 * 3
    net = iim.Network(bf16=True, seed=0)
    losses = rec.warm_start_train(net, iters=2000, batch=64, lr=1e-3, seed=1)
    assert np.all(np.isfinite(losses))
    assert losses[-100:].mean() < 0.25 * losses[:100].mean(), (losses[:100].mean(), losses[-100:].mean())

    om0, G0 = _state(w, geo, 0)
    steps = 20
    out = {}
    for name, mode in (("previous", iim.GUESS_PREVIOUS), ("extrapolate", iim.GUESS_EXTRAPOLATE),
                       ("network", iim.GUESS_NETWORK)):
        ctx = iim.Context(w.grid, w.bodies, tol=1e-10, guess=mode)
        if mode == iim.GUESS_NETWORK:
            ctx.set_warm_start(mode, net)
        out[name] = _run(ctx, om0, G0, w.dt, steps) + (ctx.warm_start_stats(),)
    # from the fourth solve on, every mode has its history
    it = {k: v[2][3:].mean() for k, v in out.items()}
    r0 = {k: np.median(v[3][3:]) for k, v in out.items()}
    print("iterations", it, "initial residuals", r0, "network", out["network"][4])
    assert r0["extrapolate"] < 0.5 * r0["previous"], r0
    assert r0["network"] < 0.8 * r0["extrapolate"], r0
    assert it["extrapolate"] < it["previous"] - 1.0, it
    assert it["network"] < it["previous"] + 1.0, it
    st = out["network"][4]
    assert st["net_used"] > 10 * st["net_rejected"], st
    # the guess changes the iterations, not the answer
    ref = ONS.Stepper(geo)
    om = np.where(geo.fluid, om0, 0.0)
    G = np.array(G0, dtype=np.float64)
    for _ in range(steps):
        om, G = ref.step(om, G, w.dt)
    for k, v in out.items():
        e = rel(v[0], om, mask=geo.fluid)
        assert e < 1e-8, (k, e)


def test_binding_refuses_mismatched_shapes():
    """x, seq and the output or target must agree in batch and length: the
    binding raises before any kernel can read or write past a buffer."""
    sizes = SIZES["small"]
    X, T, params, flat = _case(sizes, [40, 24], B=2, seed=3)
    net = iim.Network(in_channels=sizes[0], width=sizes[1], layers=len(sizes) - 1, bf16=False)
    seq = torch.as_tensor(_segments([40, 24]), device=DEV)
    x, t = _dev32(X), _dev32(T)
    y = torch.zeros((X.shape[0], X.shape[1]), dtype=torch.float32, device=DEV)
    for args in ((x, seq[:, :-1], y), (x, seq, y[:, :-1]), (x, seq, y[:1]), (x[:, :, :-1], seq, y), (x[0], seq, y)):
        with pytest.raises(ValueError):
            net.forward(*args)
    with pytest.raises(ValueError):
        net.grad_mse(x, seq, t[:, :-1])
    net.forward(x, seq, y)              # the consistent call still runs
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    net.close()


def test_learned_guess_on_a_held_out_reynolds_number():
    """The learned-guess protocol of the benchmark at a small size: runs of
    the small cylinder at four Reynolds numbers (centres moved by sub-cell
    offsets) train one network, a fifth validates (the best of six chunks is
    kept), and the run at Re 100 with the centred body, never seen, is
    solved to 1e-10 with each guess.  Asserted: the extrapolated guess needs
    fewer Krylov iterations than the previous-stage guess; the network's
    correction of it needs no more than the extrapolation (measured here
    12.93 against 13.02 per solve; on the benchmark's runs of the 1024 x 512
    cylinder 7.6 against 8.4); the guess does not change the answer."""
    base = wl.cylinder_small()
    g0 = base.grid

    def run_ctx(re, dx, dy, solver=iim.SOLVER_DIRECT, **kw):
        w = wl.cylinder(nx=g0.nx, ny=g0.ny, h=g0.h, points=128, dt=base.dt, center=(1.5 + dx, dy), nu=1.0 / re)
        return w, iim.Context(w.grid, w.bodies, solver=solver, **kw)

    rng = np.random.default_rng(3)
    ctxs = {}
    for re in (60, 90, 120, 150, 250):
        dx, dy = rng.uniform(-0.5, 0.5, 2) * g0.h
        w, c = run_ctx(re, dx, dy)
        c.record_solves(3 * 150)
        om = torch.zeros((g0.ny, g0.nx), dtype=torch.float64, device=DEV)
        c.rk3_steps(om, np.zeros(c.n_circ), w.dt, 150)
        ctxs[re] = c
    torch.cuda.synchronize()
    train = [ctxs[r] for r in (60, 90, 150, 250)]
    net = iim.Network(bf16=True, seed=0)
    best = (np.inf, None)
    for chunk in range(6):
        iim.warm_start_train_multi(train, net, iters=250, batch=32, lr=1e-3, seed=10 + chunk)
        vl, _ = ctxs[120].warm_start_loss(net)
        if vl < best[0]:
            best = (vl, net.get())
    net.set(best[1])
    for c in ctxs.values():
        c.close()
    w, spin = run_ctx(100.0, 0.0, 0.0)
    om0 = torch.zeros((g0.ny, g0.nx), dtype=torch.float64, device=DEV)
    G0, _ = spin.rk3_steps(om0, np.zeros(spin.n_circ), w.dt, 40)
    torch.cuda.synchronize()
    spin.close()
    out = {}
    for name, mode in (("previous", iim.GUESS_PREVIOUS), ("extrapolate", iim.GUESS_EXTRAPOLATE),
                       ("network", iim.GUESS_NETWORK)):
        _, ctx = run_ctx(100.0, 0.0, 0.0, solver=iim.SOLVER_KRYLOV, tol=1e-10, guess=mode)
        if mode == iim.GUESS_NETWORK:
            ctx.set_warm_start(mode, net)
        om = om0.clone()
        G = np.array(G0, dtype=np.float64)
        its = []
        for k in range(23):
            G, st = ctx.rk3_steps(om, G, w.dt, 1)
            if k >= 3:
                its += st["iters"]
        torch.cuda.synchronize()
        out[name] = (np.mean(its), om.cpu().numpy(), G)
        ctx.close()
    it = {k: v[0] for k, v in out.items()}
    print("held-out Re 100: iterations per solve", it, "validation loss", best[0])
    assert it["extrapolate"] < it["previous"], it
    assert it["network"] <= it["extrapolate"] + 0.25, it
    ref = out["previous"][1]
    for k in ("extrapolate", "network"):
        assert rel(out[k][1], ref) < 1e-8, k
    net.close()
