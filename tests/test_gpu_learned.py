"""Learned initial density on the GPU against the oracle (runs on an
MI355X): the bf16 MFMA GEMM, the MLP forward and gradient, the sample
features, the spherical-harmonic basis and transfers, and the effect of a
trained network on GMRES."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import learned as OL  # noqa: E402
from paper_2309_05965_amd import workloads as W  # noqa: E402


def bf16_bits(x):
    """bf16 bit patterns (round to nearest even) of a float array, as int16."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16)).cuda()


@pytest.mark.parametrize("shape", [(70, 50, 45), (64, 64, 32), (256, 256, 9216), (130, 1024, 256), (72, 136, 40),
                                   (2048, 324, 256)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
def test_gemm_bf16_matches_float64_of_rounded_operands(shape, ta, tb):
    from paper_2309_05965_amd import learned
    M, N, K = shape
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C = learned.gemm_bf16(bf16_bits(A), bf16_bits(B), ta, tb).cpu().numpy()
    Ar, Br = OL.bf16(A), OL.bf16(B)
    ref = (Ar.T if ta else Ar) @ (Br.T if tb else Br)
    scale = np.abs(Ar.T if ta else Ar) @ np.abs(Br.T if tb else Br)
    assert np.max(np.abs(C - ref) / scale) < 1e-6


def test_real_sh_matches_oracle():
    from paper_2309_05965_amd import learned
    d = np.random.default_rng(0).standard_normal((300, 3))
    d[0] = [0.0, 0.0, 1.0]
    d[1] = [0.0, 0.0, -2.0]
    Y = learned.real_sh(torch.from_numpy(d).cuda()).cpu().numpy().T
    assert np.max(np.abs(Y - OL.real_sh(d))) < 1e-12


def test_features_match_oracle():
    from paper_2309_05965_amd import learned
    S = W.fibonacci_sphere()
    geoms, jumps, ref = [], [], []
    for seed in (1, 2, 3):
        prob, geom, jmp = W.config5(seed, N=64)
        geoms.append(learned.pack_geometry(geom))
        jumps.append(learned.pack_jumps(jmp))
        ref.append(OL.features(geom, lambda X, j=jmp: W.jump_values(j, X), S).reshape(-1))
    X = learned.features(torch.tensor(np.array(geoms)).cuda(), torch.tensor(np.array(jumps)).cuda(),
                         torch.from_numpy(S).cuda()).cpu().numpy()
    ref = np.array(ref)
    assert np.max(np.abs(X - ref) / (1 + np.abs(ref))) < 1e-6


def test_transfers_match_oracle():
    from paper_2309_05965_amd import kfbi, learned
    prob, geom, jmp = W.config5(4, N=64)
    gp = kfbi.Plan(prob)
    S = W.fibonacci_sphere()
    dof_pos = gp.export("dof_pos").cpu().numpy()
    rng = np.random.default_rng(5)
    psi_s = rng.standard_normal(S.shape[0]).astype(np.float32)
    g = torch.tensor(learned.pack_geometry(geom)).cuda()
    St = torch.from_numpy(S).cuda()
    out = learned.transfer(gp, g, St, torch.from_numpy(psi_s).cuda(), 2.0).cpu().numpy()
    ref = OL.transfer_to_dofs(geom, S, 2.0 * psi_s.astype(np.float64), dof_pos)
    assert np.max(np.abs(out - ref)) < 1e-9 * (1 + np.max(np.abs(ref)))
    psi_d = rng.standard_normal(gp.n_dof)
    out = learned.sample(gp, g, torch.from_numpy(psi_d).cuda(), St, 0.5).cpu().numpy()
    ref = 0.5 * OL.sample_density(geom, S, dof_pos, psi_d)
    assert np.max(np.abs(out - ref)) < 1e-5 * (1 + np.max(np.abs(ref)))


def _small_mlp(widths, seed):
    from paper_2309_05965_amd import learned
    m = learned.MLP(widths)
    rng = np.random.default_rng(seed)
    p = np.zeros(m.n_params, dtype=np.float32)
    Ws, bs = [], []
    for ow, (a, b), ob, nb in m.layout():
        Wl = (rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32)
        bl = (rng.standard_normal(b) * 0.1).astype(np.float32)
        p[ow:ow + a * b] = Wl.ravel()
        p[ob:ob + nb] = bl
        Ws.append(Wl.astype(np.float64))
        bs.append(bl.astype(np.float64))
    m.set_params(torch.from_numpy(p).cuda())
    return m, Ws, bs


U32 = 2.0 ** -24


def _near_midpoint(x, e):
    """Where bf16(x) may round the other way when x moves by up to e: x
    within e of the midpoint between its two neighbouring bf16 values."""
    x = np.asarray(x, dtype=np.float64)
    lo = OL.bf16(x)
    half = np.maximum(np.abs(lo) * 2.0 ** -8, np.abs(x) * 2.0 ** -9)
    return np.abs(np.abs(x - lo) - half) <= e


def _error_bounds(Ws, bs, X, Y, C=None):
    """Worst-case elementwise bounds of the GPU's forward output and
    gradients against the bf16-emulating oracle.  Both sides round the same
    fp32 inputs and masters to bf16; they differ in the accumulation (fp32
    against fp64: at most K u sum |terms| for K terms, u = 2^-24), and an
    intermediate that lies within its error bound of a bf16 rounding
    midpoint may round one unit (2^-8 relative) the other way.  A hidden
    pre-activation within its error bound of zero may fall on either side
    of the ReLU: its back-propagated value is then da or 0.  Worst-case
    bounds compound with depth, so they are useful for small networks."""
    r = OL.bf16
    a, zs = OL.mlp_forward(Ws, bs, X, emulate=True)
    L = len(Ws)
    ea = np.zeros_like(a[0])
    fa = np.zeros(a[0].shape, dtype=bool)
    EA, FA, EZ = [ea], [fa], []
    for l in range(L):
        ra, rw = np.abs(r(a[l])), np.abs(r(Ws[l]))
        e = Ws[l].shape[0] * U32 * (ra @ rw + np.abs(bs[l])) + (2.0 ** -8 * fa * ra + ea) @ rw
        EZ.append(e)
        if l < L - 1:
            ea, fa = e, _near_midpoint(a[l + 1], e)
            EA.append(ea)
            FA.append(fa)
    out, eout = a[-1], EZ[-1]
    if C is not None:
        # linear head in fp32: y[k] = sum_j C_j z[j K + k]
        C = np.asarray(C, dtype=np.float64)
        nb = C.shape[1]
        K = out.shape[1] // nb
        z3 = out.reshape(-1, nb, K)
        e3 = eout.reshape(-1, nb, K)
        y = np.einsum("bj,bjk->bk", C, z3)
        ey = nb * U32 * np.einsum("bj,bjk->bk", np.abs(C), np.abs(z3)) + np.einsum("bj,bjk->bk", np.abs(C), e3)
        n = y.size
        dy = 2.0 * (y - np.asarray(Y, dtype=np.float64)) / n
        edy = 2.0 * ey / n + U32 * np.abs(dy)
        dz = (C[:, :, None] * dy[:, None, :]).reshape(out.shape)
        edz = (np.abs(C)[:, :, None] * (edy[:, None, :] + U32 * np.abs(dy)[:, None, :])).reshape(out.shape)
        out, eout = y, ey
    else:
        n = out.size
        dz = 2.0 * (out - np.asarray(Y, dtype=np.float64)) / n
        edz = 2.0 * eout / n
    gW_b, gb_b = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        fdz = _near_midpoint(dz, edz)
        ra, rdz = np.abs(r(a[l])), np.abs(r(dz))
        gW_b[l] = (dz.shape[0] * U32 * ra.T @ rdz + (2.0 ** -8 * FA[l] * ra + EA[l]).T @ rdz
                   + ra.T @ (2.0 ** -8 * fdz * rdz + edz))
        gb_b[l] = dz.shape[0] * U32 * np.abs(dz).sum(axis=0) + edz.sum(axis=0)
        if l > 0:
            rw = np.abs(r(Ws[l]))
            da = r(dz) @ r(Ws[l]).T
            eda = Ws[l].shape[1] * U32 * rdz @ rw.T + (2.0 ** -8 * fdz * rdz + edz) @ rw.T
            amb = np.abs(zs[l - 1]) <= EZ[l - 1]
            on = zs[l - 1] > 0.0
            dz = da * on
            edz = np.where(amb, np.abs(da) + eda, np.where(on, eda, 0.0))
    return out, eout, gW_b, gb_b


@pytest.mark.parametrize("widths,B", [((40, 24, 24, 16), 20), ((9216, 256, 256, 256, 1024), 64),
                                      ((40, 24, 24, 16), 3), ((9216, 256, 256, 256, 1024), 1),
                                      ((15, 24, 24, 16), 1000), ((15, 256, 256, 256, 324), 2048)])
def test_mlp_forward_and_gradient_match_oracle(widths, B):
    """Small network: forward output and every gradient entry within the
    worst-case bounds of _error_bounds.  Full-size network (where those
    bounds compound to uselessness): 99% of the entries within 1e-3 of
    their size plus 1e-3 of the layer's rms (ReLU gates that sit at zero
    to rounding may switch), and the relative difference in norm below
    1e-2."""
    m, Ws, bs = _small_mlp(widths, 7)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((B, widths[0])).astype(np.float32)
    Y = rng.standard_normal((B, widths[-1])).astype(np.float32)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = m.forward(Xt).cpu().numpy()
    loss, g = m.loss_grad(Xt, Yt)
    lref, gW, gb = OL.mlp_loss_grad(Ws, bs, X, Y, emulate=True)
    assert float(loss.item()) == pytest.approx(lref, rel=1e-3)
    g = g.cpu().numpy()
    small = max(widths) < 100
    if small:
        ref, ob, gWb, gbb = _error_bounds(Ws, bs, X, Y)
        assert np.all(np.abs(out - ref) <= ob)
    else:
        ref = OL.mlp_forward(Ws, bs, X, emulate=True)[0][-1]
        assert np.linalg.norm(out - ref) <= 1e-2 * np.linalg.norm(ref)
    for l, (ow, (i, o), ob_, nb) in enumerate(m.layout()):
        dW = g[ow:ow + i * o].reshape(i, o)
        db = g[ob_:ob_ + nb]
        if small:
            assert np.all(np.abs(dW - gW[l]) <= gWb[l]), l
            assert np.all(np.abs(db - gb[l]) <= gbb[l]), l
            # the bounds stay well below the gradient for most entries
            nz = gW[l] != 0.0
            assert np.mean((gWb[l] < 0.1 * np.abs(gW[l]))[nz]) > 0.75
        else:
            for got, want in ((dW, gW[l]), (db, gb[l])):
                rms = np.sqrt(np.mean(want * want))
                r = np.abs(got - want) / (np.abs(want) + rms)
                print("layer %d: relative differences, median %.1e, 99%% %.1e, max %.1e"
                      % (l, np.median(r), np.quantile(r, 0.99), r.max()))
                assert np.quantile(r, 0.99) <= 5e-2, l
                assert np.linalg.norm(got - want) <= 1e-2 * np.linalg.norm(want)


def test_adam_steps_match_oracle():
    """Two Adam steps of the GPU (forward, backward and update in one call
    each) against the oracle's gradient and Adam update: where the oracle's
    gradient is clear of its error bound, every parameter moves by the
    oracle's step to 1e-3 of the learning rate; elsewhere by at most the
    step bound lr / sqrt(1 - b2) of Adam's first two steps."""
    widths, B, lr = (40, 24, 24, 16), 20, 1e-4
    m, Ws, bs = _small_mlp(widths, 7)
    p0 = m.get_params().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((B, widths[0])).astype(np.float32)
    Y = rng.standard_normal((B, widths[-1])).astype(np.float32)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    lay = m.layout()

    def pack(gW, gb):
        out = np.zeros(m.n_params)
        for l, (ow, (i, o), ob, nb) in enumerate(lay):
            out[ow:ow + i * o] = gW[l].ravel()
            out[ob:ob + nb] = gb[l]
        return out

    def unpack(p):
        return ([p[ow:ow + i * o].reshape(i, o) for ow, (i, o), ob, nb in lay],
                [p[ob:ob + nb] for ow, (i, o), ob, nb in lay])

    pr, mm, vv = p0, np.zeros(m.n_params), np.zeros(m.n_params)
    prev = p0
    clear = np.ones(m.n_params, dtype=bool)
    for t in (1, 2):
        Wr, br = unpack(pr)
        _, gW, gb = OL.mlp_loss_grad(Wr, br, X, Y, emulate=True)
        _, _, gWb, gbb = _error_bounds(Wr, br, X, Y)
        g, gbound = pack(gW, gb), pack(gWb, gbb)
        # entries whose gradient is clear of its bound, or exactly zero on
        # both sides (a zero bound: no term can differ)
        clear &= (np.abs(g) > 10.0 * gbound + 1e-6) | ((gbound == 0.0) & (g == 0.0))
        pr, mm, vv = OL.adam_step(pr, g, mm, vv, t, lr)
        m.train_step(Xt, Yt, lr)
        pg = m.get_params().cpu().numpy().astype(np.float64)
        step_g, step_r = pg - prev, pr - (prev if t == 1 else prev_r)
        assert clear.mean() > 0.8
        # 1e-3 lr, plus the fp32 rounding of the updated master weight
        assert np.all(np.abs(step_g - step_r)[clear] <= 1e-3 * lr + 1.5 * U32 * np.abs(prev[clear]))
        assert np.all(np.abs(step_g) <= lr / np.sqrt(1 - 0.999) * 1.01)
        prev, prev_r = pg, pr
        # the GPU continues from its own parameters; the oracle from its own


def test_training_reduces_the_loss():
    m, _, _ = _small_mlp((32, 64, 64, 8), 3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, 32)).astype(np.float32)
    T = rng.standard_normal((32, 8)) / 6
    Y = np.tanh(X @ T).astype(np.float32)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    first = m.loss_grad(Xt, Yt)[0].item()
    for _ in range(300):
        m.train_step(Xt, Yt, 3e-3)
    last = m.loss_grad(Xt, Yt)[0].item()
    assert last < 0.1 * first


def test_pretrained_warm_start_gains_on_heldout_seeds():
    """The stored network (trained on solver densities of N = 128
    ellipsoids) predicts held-out densities to well under the zero start's
    100% error, saves GMRES iterations, and the whole solve including the
    prediction takes less time than the solve from the zero start; every
    solve still reaches the tolerance."""
    import time
    from paper_2309_05965_amd import kfbi, learned, warmstart
    model = warmstart.load_pretrained()
    zero, learn, err_l, tz, tl = [], [], [], [], []
    plan = None
    for seed in range(1_000_100, 1_000_116):
        prob, geom, jmp = W.config5(seed, 128)
        try:
            if plan is None:
                plan = kfbi.Plan(prob)
            else:
                plan.setup(prob)
        except kfbi.KfbiError:
            plan = None
            continue
        d = kfbi.device_jump_data(plan, jmp)
        ref, _, _ = plan.solve(d, tol=1e-11)
        best_z, best_l = np.inf, np.inf
        for _ in range(3):                          # best of three of each (graph warm-up included)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, iz = plan.solve(d, tol=1e-8)
            torch.cuda.synchronize()
            best_z = min(best_z, time.perf_counter() - t)
            t = time.perf_counter()
            p0 = warmstart.predict(model, plan, geom, jmp)
            _, _, il = plan.solve(d, tol=1e-8, psi0=p0)
            torch.cuda.synchronize()
            best_l = min(best_l, time.perf_counter() - t)
            # the same start predicted inside the solve (kfbi_opts)
            psi_o, _, io = plan.solve(d, tol=1e-8, learned=warmstart.learned_args(model, geom, jmp))
            assert io["iters"] == il["iters"] and io["status"] == 0
        assert il["status"] == 0 and il["true_rel_res"] < 2e-8
        zero.append(iz["iters"])
        learn.append(il["iters"])
        tz.append(best_z)
        tl.append(best_l)
        err_l.append(float(((p0 - ref).norm() / ref.norm()).item()))
    print("iters zero %.2f learned %.2f; density error %.3f; solve ms zero %.2f learned %.2f"
          % (np.mean(zero), np.mean(learn), np.mean(err_l), 1e3 * np.mean(tz), 1e3 * np.mean(tl)))
    assert len(zero) >= 12
    assert np.mean(err_l) < 0.25
    assert np.mean(learn) < np.mean(zero) - 1.0
    assert np.sum(tl) < np.sum(tz)


def test_linear_head_matches_oracle():
    """The linear head (density linear in the jump coefficients): forward
    output and every gradient entry of a small network within the
    worst-case bounds of _error_bounds with the head."""
    widths, B, nb = (15, 24, 24, 3 * 4), 20, 3
    m, Ws, bs = _small_mlp(widths, 11)
    rng = np.random.default_rng(12)
    X = rng.standard_normal((B, widths[0])).astype(np.float32)
    C = rng.standard_normal((B, nb)).astype(np.float32)
    Y = rng.standard_normal((B, widths[-1] // nb)).astype(np.float32)
    Xt, Ct, Yt = (torch.from_numpy(v).cuda() for v in (X, C, Y))
    out = m.forward_lin(Xt, Ct, nb).cpu().numpy()
    ref, ob, gWb, gbb = _error_bounds(Ws, bs, X, Y, C)
    assert np.all(np.abs(out - ref) <= ob)
    loss, g = m.loss_grad_lin(Xt, Ct, nb, Yt)
    lref, gW, gb = OL.mlp_lin_loss_grad(Ws, bs, X, C, Y, emulate=True)
    assert float(loss.item()) == pytest.approx(lref, rel=1e-4)
    g = g.cpu().numpy()
    for l, (ow, (i, o), ob_, nbias) in enumerate(m.layout()):
        assert np.all(np.abs(g[ow:ow + i * o].reshape(i, o) - gW[l]) <= gWb[l]), l
        assert np.all(np.abs(g[ob_:ob_ + nbias] - gb[l]) <= gbb[l]), l


def test_sh_coefficients_and_expansion_match_oracle():
    from paper_2309_05965_amd import kfbi, learned
    prob, geom, jmp = W.config5(4, N=64)
    gp = kfbi.Plan(prob)
    dof_pos = gp.export("dof_pos").cpu().numpy()
    rng = np.random.default_rng(6)
    psi = rng.standard_normal(gp.n_dof)
    g = torch.tensor(learned.pack_geometry(geom)).cuda()
    coef = learned.sh_coefficients(gp, g, torch.from_numpy(psi).cuda(), 0.5).cpu().numpy()
    ref = 0.5 * OL.sh_coefficients(geom, dof_pos, psi)
    assert np.max(np.abs(coef - ref)) <= 1e-9 * np.max(np.abs(ref))
    c2 = rng.standard_normal(81)
    vals = learned.sh_expand(gp, g, torch.from_numpy(c2).cuda(), 2.0).cpu().numpy()
    assert np.max(np.abs(vals - 2.0 * OL.sh_values(geom, dof_pos, c2))) <= 1e-12 * np.max(np.abs(vals))


def test_learned_start_pipeline_matches_oracle():
    """kfbi_learned_start (geometry input, network, linear head with the
    jump coefficients, harmonics at the DOFs) against the oracle's steps
    with a random network of the stored model's shape."""
    from paper_2309_05965_amd import kfbi, learned, warmstart
    widths = warmstart.WIDTHS
    m, Ws, bs = _small_mlp(widths, 13)
    prob, geom, jmp = W.config5(5, N=64)
    gp = kfbi.Plan(prob)
    g = torch.tensor(learned.pack_geometry(geom)).cuda()
    j = torch.tensor(learned.pack_jumps(jmp)).cuda()
    psi = learned.learned_start(gp, m, warmstart.NB, g, j, 0.7).cpu().numpy()
    x = OL.mode_rows(geom).astype(np.float32)
    Xg = learned.geometry_input(g[None, :]).cpu().numpy()
    assert np.max(np.abs(Xg - x)) <= 1e-6 * np.max(np.abs(x))
    z = OL.mlp_forward(Ws, bs, x, emulate=True)[0][-1].reshape(1, -1)
    coef = 0.7 * OL.lin_head(z, OL.mode_major(learned.pack_jumps(jmp))[None, :], warmstart.NB)[0]
    ref = OL.sh_values(geom, gp.export("dof_pos").cpu().numpy(), coef)
    # fp32 accumulation in the network (about 1e-6 of its sums) against fp64
    assert np.max(np.abs(psi - ref)) <= 1e-3 * np.max(np.abs(ref))


def test_linear_head_rows_per_example():
    """R rows per example: the head reads an example's R rows as one row
    (forward and loss against the oracle, FP32 accumulation)."""
    widths, B, R, nb = (15, 24, 24, 8), 6, 4, 8
    m, Ws, bs = _small_mlp(widths, 14)
    rng = np.random.default_rng(15)
    X = rng.standard_normal((B * R, widths[0])).astype(np.float32)
    C = rng.standard_normal((B, nb)).astype(np.float32)
    Y = rng.standard_normal((B, R * widths[-1] // nb)).astype(np.float32)
    Xt, Ct, Yt = (torch.from_numpy(v).cuda() for v in (X, C, Y))
    out = m.forward_lin(Xt, Ct, nb, R).cpu().numpy()
    z = OL.mlp_forward(Ws, bs, X, emulate=True)[0][-1].reshape(B, -1)
    ref = OL.lin_head(z, C, nb)
    assert np.max(np.abs(out - ref)) <= 1e-4 * np.max(np.abs(ref))
    loss, _ = m.loss_grad_lin(Xt, Ct, nb, Yt, R)
    lref, _, _ = OL.mlp_lin_loss_grad(Ws, bs, X, C, Y, emulate=True, R=R)
    assert float(loss.item()) == pytest.approx(lref, rel=1e-4)
