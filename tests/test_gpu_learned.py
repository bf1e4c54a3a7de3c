"""GPU parity of the learned preconditioner stage: the matrix-core
convolution kernels (forward, input gradient, weight gradient) against the
FP64 convolution on the same BF16 operands, the whole correction map and
the training loss/gradient against the BF16-storage oracle, the harvested
training pairs against the oracle's V-cycle, and the flexible-CG solver
(with zero, random and non-finite weights) against the FP64 oracle.

Bars: a convolution layer is within the FP32 summation bound
n u sum|terms| (n the number of terms summed one after another, u = 2^-24);
the whole network and its gradients, where an accumulation-order change
can move a BF16 rounding of an intermediate activation, within 1e-3
relative L2; solves as for the FP64 path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W
from oracle import learned, nn, solvers
from oracle.grid import Grid
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
TIGHT = 1e-12


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _layers(flat):
    out, o = [], 0
    for co, ci in ibpm.NN_SHAPES:
        out.append(np.asarray(flat[o:o + co * ci * 9], dtype=np.float64).reshape(co, ci, 3, 3))
        o += co * ci * 9
    return out


def _hwc(x):            # (C, H, W) -> (H, W, C)
    return np.ascontiguousarray(np.transpose(x, (1, 2, 0)))


def _chw(x, ny, nx, c):
    return np.transpose(np.asarray(x).reshape(ny, nx, c), (2, 0, 1))


# ragged in x (136 = 128 + 8 pixels: two tiles of a row, the second nearly empty)
LAYER_WL = lambda: W.tiny(136, 72, 12, radius=0.3)
# stretched grid, 160 x 160 (two tiles per row), body on the uniform patch
NET_WL = lambda: W.cylinder_stretched(160, 0.05, 40, 40.0, 0.01, 2)


@pytest.mark.parametrize("layer", [0, 1, 5])
def test_conv_layer_kernels_match_fp64_convolution(layer):
    wl = LAYER_WL()
    print(f"[nn layer] {layer} {wl.nx}x{wl.ny}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1)
    ctx.nn_init(seed=100 + layer)
    Wl = nn.bf16_round(_layers(ctx.nn_get_weights())[layer])
    co, ci = ibpm.NN_SHAPES[layer]
    cin = 8 if layer == 0 else 32
    rng = np.random.default_rng(layer)
    ny, nx = wl.ny, wl.nx
    x = np.zeros((cin, ny, nx))
    x[:ci] = nn.bf16_round(rng.standard_normal((ci, ny, nx)))
    xt = _t(_hwc(x), torch.float32)
    # forward
    y = _chw(_n(ctx.nn_layer(layer, 0, x=xt)), ny, nx, 32)
    ref = nn.conv3x3(x[:ci], Wl)
    bound = 9 * ci * U * nn.conv3x3(np.abs(x[:ci]), np.abs(Wl)) + 1e-30
    assert np.all(np.abs(y[:co] - ref) <= bound)
    assert np.all(y[co:] == 0.0)
    # input gradient through a ReLU mask
    dy = np.zeros((32, ny, nx))
    dy[:co] = rng.standard_normal((co, ny, nx))
    mask = np.where(rng.random((32, ny, nx)) < 0.5, 1.0, -1.0)
    g = nn.bf16_round(dy * (mask > 0))
    dx = _chw(_n(ctx.nn_layer(layer, 1, dy=_t(_hwc(dy), torch.float32),
                              mask=_t(_hwc(mask), torch.float32))), ny, nx, 32)
    ref = nn.conv3x3_grad_input(g[:co], Wl)
    bound = 9 * co * U * nn.conv3x3_grad_input(np.abs(g[:co]), np.abs(Wl)) + 1e-30
    assert np.all(np.abs(dx[:ci] - ref) <= bound)
    # weight gradient: per tile the matrix cores sum 128 pixels in 8 steps,
    # then the tiles (2 per row, 72 rows) are added one after another
    dw = _n(ctx.nn_layer(layer, 2, x=xt, dy=_t(_hwc(dy), torch.float32),
                         mask=_t(_hwc(mask), torch.float32))).reshape(co, ci, 3, 3)
    ref = nn.conv3x3_grad_weight(x[:ci], g[:co])
    nsum = 128 + 2 * ny
    bound = nsum * U * nn.conv3x3_grad_weight(np.abs(x[:ci]), np.abs(g[:co])) + 1e-30
    assert np.all(np.abs(dw - ref) <= bound)
    print(f"  fwd/dx/dw within the summation bound", flush=True)
    ctx.close()


def test_network_correction_matches_bf16_oracle():
    wl = NET_WL()
    print(f"[nn apply] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1)
    ctx.nn_init(seed=7)
    ws = _layers(ctx.nn_get_weights())
    g = Grid(wl.xf, wl.yf)
    D = learned.cell_delta(g, wl.xb, wl.yb)
    r = W.random_vector(ctx.n_lambda, 21) * 3e-4
    e = _n(ctx.nn_apply(_t(r)))
    ref = learned.apply(g, D, ws, r, wl.dt)
    err = _rel(e, ref)
    nc = g.nx * g.ny
    ef = _rel(e[nc:], ref[nc:])
    print(f"  rel L2 {err:.2e} (forces {ef:.2e})", flush=True)
    assert err < 1e-3 and ef < 1e-3
    ctx.close()


def test_training_loss_and_gradient_match_bf16_oracle():
    wl = NET_WL()
    print(f"[nn grad] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1)
    ctx.nn_init(seed=8)
    ws = _layers(ctx.nn_get_weights())
    P = Problem(wl, poisson_solver=0)
    g = P.grid
    D = learned.cell_delta(g, wl.xb, wl.yb)
    # a consistent pair: r1 = K e1 (both as FP32)
    e1 = (W.random_vector(ctx.n_lambda, 32) * 50.0).astype(np.float32)
    r1 = (P.ops.K @ e1.astype(np.float64)).astype(np.float32)
    loss, grad = ctx.nn_loss_grad(_t(r1, torch.float32), _t(e1, torch.float32))
    rl, rg = learned.sample_loss_grad(g, D, P.ops.K, ws, r1, e1, wl.dt)
    print(f"  loss gpu {loss:.8g} oracle {rl:.8g}", flush=True)
    assert -1.0 <= rl < 0.0
    # the loss is a ratio whose numerator (d . r1)^2 is small for an untrained
    # network, so BF16-level differences in d show up relatively larger
    assert abs(loss - rl) <= 2e-3 * abs(rl)
    for l, (a, b) in enumerate(zip(_layers(grad), rg)):
        err = _rel(a, b)
        print(f"  layer {l} gradient rel L2 {err:.2e}", flush=True)
        assert err < 1e-3
    ctx.close()


def test_adam_pass_lowers_loss_and_is_deterministic():
    wl = LAYER_WL()
    print(f"[nn train] {wl.name}", flush=True)
    res = []
    for rep in range(2):
        ctx = ibpm.Context(wl, poisson_solver=1)
        ctx.nn_init(seed=3)
        e1 = torch.stack([_t(W.random_vector(ctx.n_lambda, 50 + k)) for k in range(4)])
        r1 = torch.stack([ctx.apply_K(e1[k].contiguous()) for k in range(4)])
        losses = [ctx.nn_train(r1.float().contiguous(), e1.float().contiguous(), [0, 1, 2, 3], 2, 1e-3)
                  for _ in range(15)]
        res.append((losses, ctx.nn_get_weights()))
        ctx.close()
    print(f"  losses {res[0][0][0]:.4f} -> {res[0][0][-1]:.4f}", flush=True)
    assert res[0][0][-1] < res[0][0][0]
    assert res[0][0] == res[1][0]
    np.testing.assert_array_equal(res[0][1], res[1][1])


def test_adam_steps_match_oracle():
    """The device Adam update (k_adam through ibpm_nn_adam_step) against the
    oracle's Adam step (Kingma & Ba, bias-corrected): five steps from the
    oracle's He-normal weights on a seeded sequence of gradients whose
    elements change direction and scale from step to step (so that both
    moment averages and both bias corrections enter), with two learning
    rates.  FP32 on the device, FP64 in the oracle: every weight within ten
    times the FP32 rounding of the weight and of the updates."""
    wl = LAYER_WL()
    print(f"[nn adam] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1)
    chans = [ibpm.NN_SHAPES[0][1]] + [co for co, _ in ibpm.NN_SHAPES]
    w0 = np.concatenate([x.ravel() for x in nn.init_weights(chans, 4)]).astype(np.float32)
    ctx.nn_set_weights(w0)
    w = w0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    rng = np.random.default_rng(21)
    lrs = [1e-3, 1e-3, 5e-4, 5e-4, 1e-3]
    for t, lr in enumerate(lrs, start=1):
        g = (rng.standard_normal(w.size) * 10.0 ** rng.uniform(-4, 1, w.size)).astype(np.float32)
        ctx.nn_adam_step(g, lr)
        w, m, v = nn.adam_step(w, g.astype(np.float64), m, v, t, lr)
    wg = ctx.nn_get_weights().astype(np.float64)
    ctx.close()
    # each update has |m^/(sqrt(v^)+eps)| <= a few units; FP32 evaluates it
    # to a few ulps and rounds the weight once per step
    bound = 10.0 * len(lrs) * (2.0 ** -23 * np.abs(w) + 3.0 * 2.0 ** -23 * max(lrs) * 4.0)
    worst = float(np.max(np.abs(wg - w) / bound))
    moved = float(np.median(np.abs(wg - w0)))
    print(f"  worst |w_gpu - w_oracle| / bound {worst:.3f}; median move {moved:.2e}", flush=True)
    assert worst <= 1.0
    assert moved > 1e-3


def _amg_problem():
    wl = W.cylinder_small(96, 60).replace(poisson_solver=1)
    return wl, Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)


def _realistic_rhs(P, wl, steps=2):
    st, _ = P.run(steps)
    from oracle import flow
    o = P.ops
    w1 = flow.update_walls(P.grid, st.walls, st.q, wl.uinf, wl.alpha, o.dt)
    conv = flow.convection(P.grid, st.q, st.walls)
    r1 = flow.momentum_rhs(o, st.q, conv, st.conv_prev, st.walls, w1)
    dinv = 1.0 / o.A.diagonal()
    qs, _, _ = solvers.pcg(o.apply_A, r1, st.q, lambda r: dinv * r, TIGHT, 5000)
    return flow.poisson_rhs(o, qs, w1, P.ub), st


def test_harvested_pairs_match_oracle_vcycle():
    wl, P = _amg_problem()
    print(f"[harvest] {wl.name}", flush=True)
    rhs = W.random_vector(P.ops.K.shape[0], 61)
    xstar, _, _ = P.solve_poisson(rhs, np.zeros_like(rhs), rtol=1e-13, maxit=20000)
    ctx = ibpm.Context(wl, poisson_solver=1)
    x = ctx.zeros_lambda()
    r1, e1 = ctx.harvest(_t(rhs), x, _t(xstar), 6)
    r1, e1 = _n(r1), _n(e1)
    assert r1.shape[0] == 6
    v = P.H.vcycle(rhs)
    ref_r1 = rhs - P.ops.K @ v
    ref_e1 = xstar - v
    print(f"  pair 0: r1 {_rel(r1[0], ref_r1):.2e} e1 {_rel(e1[0], ref_e1):.2e}", flush=True)
    assert _rel(r1[0], ref_r1) < 1e-6 and _rel(e1[0], ref_e1) < 1e-6
    # K e1 = r1 for every pair (x* exact to 1e-13); e1 is stored in FP32, so
    # the check is relative to the size of the terms of K e1
    absK = abs(P.ops.K)
    for k in range(6):
        gap = np.linalg.norm(P.ops.K @ e1[k] - r1[k]) / np.linalg.norm(absK @ np.abs(e1[k]))
        assert gap < 1e-6, (k, gap)
    ctx.close()


def _learned_solve(wl, rhs, lam0, weights=None, seed=None, rtol=TIGHT):
    ctx = ibpm.Context(wl, poisson_solver=3, poisson_rtol=rtol, poisson_maxit=20000)
    if weights is not None:
        ctx.nn_set_weights(weights)
    else:
        ctx.nn_init(seed)
    lam = _t(lam0)
    s = ctx.solve_poisson(_t(rhs), lam)
    out = _n(lam)
    ctx.close()
    return s, out


def test_learned_solver_matches_oracle_with_any_weights():
    wl, P = _amg_problem()
    print(f"[learned solve] {wl.name}", flush=True)
    rhs, st = _realistic_rhs(P, wl)
    ref, it_ref, _ = P.solve_poisson(rhs, st.lam, rtol=TIGHT, maxit=20000)
    o = P.ops
    R = P.grid.R_diag()
    proj = lambda lam: o.B1 * (o.Q @ lam) / R
    # zero weights: the stage adds nothing and FCG(1) is AMG-PCG
    s0, lam0 = _learned_solve(wl, rhs, st.lam, weights=np.zeros(ibpm.NN_PARAMS))
    ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=TIGHT, poisson_maxit=20000)
    lam1 = _t(st.lam)
    s1 = ctx.solve_poisson(_t(rhs), lam1)
    ctx.close()
    print(f"  zero weights: {s0['iters']} iters (AMG-PCG {s1['iters']}, oracle {it_ref}), "
          f"lambda err {_rel(lam0, ref):.2e}", flush=True)
    assert s0["relres"] <= TIGHT and s0["fallbacks"] == 0
    assert abs(s0["iters"] - s1["iters"]) <= 2
    assert _rel(lam0, ref) < 1e-10
    # random weights: the stage is a poor guess but the energy-optimal step
    # keeps the iteration convergent.  A flexible iteration with a nonlinear
    # stage stops with a residual of another direction than CG's, and K is
    # ill-conditioned (cond ~7e6 here), so lambda is compared at a residual
    # ten times smaller (at 1e-12 it lies 4e-10 from the oracle's)
    sr, lamr = _learned_solve(wl, rhs, st.lam, seed=5, rtol=TIGHT / 10)
    print(f"  random weights: {sr['iters']} iters, fallbacks {sr['fallbacks']}, "
          f"lambda err {_rel(lamr, ref):.2e}", flush=True)
    assert sr["relres"] <= TIGHT / 10 and _rel(lamr, ref) < 1e-10
    # sign-flipped weights
    ctx = ibpm.Context(wl, poisson_solver=1)
    ctx.nn_init(5)
    wneg = -ctx.nn_get_weights()
    ctx.close()
    sn, lamn = _learned_solve(wl, rhs, st.lam, weights=wneg, rtol=TIGHT / 10)
    print(f"  flipped weights: {sn['iters']} iters, fallbacks {sn['fallbacks']}, "
          f"lambda err {_rel(lamn, ref):.2e}", flush=True)
    assert sn["relres"] <= TIGHT / 10 and _rel(lamn, ref) < 1e-10
    # non-finite weights: the energy-optimal weight of a non-finite correction
    # is taken as 0, so the solve is AMG-PCG
    wnan = np.full(ibpm.NN_PARAMS, np.nan, dtype=np.float32)
    sf, lamf = _learned_solve(wl, rhs, st.lam, weights=wnan)
    print(f"  NaN weights: {sf['iters']} iters, fallbacks {sf['fallbacks']}", flush=True)
    assert sf["relres"] <= TIGHT and abs(sf["iters"] - s1["iters"]) <= 2
    assert _rel(lamf, ref) < 1e-10


def test_learned_solver_falls_back_when_the_residual_stalls():
    """The stall is forced from the host: with fcg_stall_fall = 1 the
    residual would have to reach zero within 16 iterations, so the flexible
    iteration hands over to AMG-PCG after 16 to 23 iterations (checks come
    at chunk ends), and AMG-PCG from that iterate reaches the oracle's
    solution."""
    wl, P = _amg_problem()
    print(f"[learned stall] {wl.name}", flush=True)
    rhs, st = _realistic_rhs(P, wl)
    ref, _, _ = P.solve_poisson(rhs, st.lam, rtol=TIGHT, maxit=20000)
    ctx = ibpm.Context(wl, poisson_solver=3, poisson_rtol=TIGHT, poisson_maxit=20000,
                       fcg_stall_fall=1.0)
    ctx.nn_init(5)
    lam = _t(st.lam)
    s = ctx.solve_poisson(_t(rhs), lam)
    print(f"  {s}, lambda err {_rel(_n(lam), ref):.2e}", flush=True)
    assert s["fallbacks"] == 1 and s["status"] == ibpm.IBPM_OK
    assert s["relres"] <= TIGHT and _rel(_n(lam), ref) < 1e-10
    ctx.close()


def test_learned_solver_falls_back_from_zero_on_nan():
    """A NaN right-hand side makes the flexible residual NaN; the solve hands
    over to AMG-PCG from zero, which reports IBPM_ENAN."""
    wl, P = _amg_problem()
    rhs = W.random_vector(P.ops.K.shape[0], 71)
    rhs[17] = np.nan
    ctx = ibpm.Context(wl, poisson_solver=3, poisson_rtol=TIGHT, poisson_maxit=200)
    ctx.nn_init(5)
    lam = ctx.zeros_lambda()
    s = ctx.solve_poisson(_t(rhs), lam, allow_fail=True)
    print(f"  {s}", flush=True)
    assert s["fallbacks"] == 1 and s["status"] == ibpm.IBPM_ENAN
    ctx.close()


def test_learned_trajectory_velocity_and_drag():
    wl = W.cylinder_small(96, 60).replace(poisson_solver=3)
    print(f"[learned trajectory] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=3, poisson_rtol=1e-8)
    ctx.nn_init(11)
    q, conv, lam = ctx.init_state()
    for _ in range(10):
        sm = ctx.step(q, conv, lam, 1)
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    ost, infos = P.run(10)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, ost.q / R)
    ecd = abs(sm["fx"] - infos[-1].fx) / abs(infos[-1].fx)
    print(f"  96^2 learned x 10 steps: velocity err {eu:.2e}, Cd err {ecd:.2e}", flush=True)
    assert eu < 1e-7 and ecd < 1e-6
    ctx.close()


def test_mixed_learned_trajectory_velocity_and_drag():
    """FP32 inner flexible CG with the learned stage inside FP64 refinement:
    fields within 1e-7 and drag within 1e-6 of the FP64 oracle."""
    wl = W.cylinder_small(96, 60).replace(poisson_solver=4)
    print(f"[mixed+learned trajectory] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=4, poisson_rtol=1e-8)
    ctx.nn_init(11)
    q, conv, lam = ctx.init_state()
    for _ in range(10):
        sm = ctx.step(q, conv, lam, 1)
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    ost, infos = P.run(10)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, ost.q / R)
    ecd = abs(sm["fx"] - infos[-1].fx) / abs(infos[-1].fx)
    print(f"  96^2 mixed+learned x 10 steps: velocity err {eu:.2e}, Cd err {ecd:.2e}, "
          f"Poisson iters/step {sm['poisson_iters'] / 10:.1f}", flush=True)
    assert sm["poisson_relres_max"] <= 1e-8
    assert eu < 1e-7 and ecd < 1e-6
    ctx.close()


WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(ibpm.__file__), "weights", "cylinder_512.npy")


def test_trained_network_gain_on_held_out_flow():
    """What the trained network gains: on a flow it was not trained on (the
    512^2 Re 40 cylinder; training used Re 100 flows of the same grid at other
    inflow angles) the trained stage removes a clear share of the energy-norm
    error that the V-cycle leaves, an untrained one almost none.  The solver
    with the trained stage still meets the 1e-8 residual with the same
    solution (iterations and fallbacks are reported, not gated)."""
    from paper_1109_3524_amd.train_learned import poisson_rhs
    w = np.load(WEIGHTS)
    wl = W.cylinder_512()
    print(f"[learned gain] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1)
    q, conv, lam = ctx.init_state()
    ctx.step(q, conv, lam, 6)
    rhs = poisson_rhs(ctx, q, conv, lam)
    lam0 = lam.clone()
    ref = lam0.clone()
    s1 = ctx.solve_poisson(rhs, ref)
    tight = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-12, poisson_maxit=20000)
    xstar = lam0.clone()
    tight.solve_poisson(rhs, xstar)
    tight.close()
    r1, e1 = ctx.harvest(rhs, lam0.clone(), xstar, 240)
    idx = list(range(0, r1.shape[0], 20))
    gains = {}
    for name, weights in (("trained", w), ("untrained", None)):
        if weights is None:
            ctx.nn_init(5)
        else:
            ctx.nn_set_weights(weights)
        gains[name] = -np.mean([ctx.nn_loss_grad(r1[k].contiguous(), e1[k].contiguous())[0] for k in idx])
    ctx.close()
    print(f"  share of the energy error removed per application: trained {gains['trained']:.3f}, "
          f"untrained {gains['untrained']:.3f} ({len(idx)} held-out pairs)", flush=True)
    assert gains["trained"] > 0.1 and gains["trained"] > 5 * gains["untrained"]
    c = ibpm.Context(wl, poisson_solver=3)
    c.nn_set_weights(w)
    x = lam0.clone()
    st = c.solve_poisson(rhs, x)
    c.close()
    print(f"  AMG-PCG {s1['iters']} iterations; with the trained stage {st['iters']} "
          f"(fallbacks {st['fallbacks']})", flush=True)
    assert st["relres"] <= 1e-8
    P = Problem(wl, poisson_solver=1)
    o = P.ops
    R = P.grid.R_diag()
    du = _rel(o.B1 * (o.Q @ _n(x)) / R, o.B1 * (o.Q @ _n(ref)) / R)
    print(f"  projection difference to AMG-PCG: {du:.2e}", flush=True)
    assert du < 1e-6


@pytest.mark.xfail(reason="the trained stage does not bring the solve below plain AMG-PCG in time: a "
                          "network application costs about as much as an AMG-PCG iteration and the "
                          "flexible recurrence needs more iterations than CG", strict=False)
def test_learned_stage_end_to_end_against_plain():
    """End to end: the time of one 512^2 Poisson solve (step 6 of the Re 40
    flow, from the previous lambda, 1e-8) with the trained stage in FCG(m)
    against plain AMG-PCG, over the stage's schedule (every k-th application)
    and the depth m of the flexible recurrence; the best setting is gated
    against plain."""
    from paper_1109_3524_amd.train_learned import poisson_rhs
    w = np.load(WEIGHTS)
    wl = W.cylinder_512()
    ctx = ibpm.Context(wl, poisson_solver=1)
    q, conv, lam = ctx.init_state()
    ctx.step(q, conv, lam, 6)
    rhs = poisson_rhs(ctx, q, conv, lam)
    lam0 = lam.clone()

    def timed(c):
        x = lam0.clone()
        c.solve_poisson(rhs, x)           # records the graphs
        x = lam0.clone()
        st = c.solve_poisson(rhs, x)
        assert st["relres"] <= 1e-8
        return st

    plain = timed(ctx)
    ctx.close()
    rows = []
    for every in (1, 2, 4):
        for depth in (1, 4, 8):
            c = ibpm.Context(wl, poisson_solver=3, learned_every=every, fcg_depth=depth)
            c.nn_set_weights(w)
            st = timed(c)
            c.close()
            rows.append((st["ms"], every, depth, st["iters"], st["fallbacks"]))
            print(f"  learned every {every} depth {depth}: {st['iters']} iterations, {st['ms']:.2f} ms, "
                  f"fallbacks {st['fallbacks']}", flush=True)
    best = min(rows)
    print(f"  plain AMG-PCG {plain['iters']} iterations, {plain['ms']:.2f} ms; best learned {best[0]:.2f} ms "
          f"(every {best[1]}, depth {best[2]})", flush=True)
    assert best[0] < plain["ms"]
