"""GPU learned preconditioner vs the FP64 oracle of the same network.

The GPU computes with BF16-rounded weights, BF16 matrix-core operands and FP32
accumulation/activations; the oracle gets the same rounded weights in FP64.
Tolerances: a BF16 operand carries a relative rounding error of at most
2^-9 ~ 2e-3; the hidden layers sum 64-96 such products per output over four
layers, and the loss is a ratio of sums, so the end-to-end error is a small
multiple of that: C to 1e-2 (norm-wise), the loss to 1e-2 relative, the
gradient to cosine >= 0.999 and 2e-2 relative norm error.
"""
import numpy as np
import pytest
import torch

from oracle import learned as LR
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float32."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def perturbed_theta(bs, seed, scale=0.05):
    theta = LR.init_params(bs, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    return (theta + scale * rng.standard_normal(theta.size)).astype(np.float32)


def factor_for(w, bs, theta):
    from paper_1805_12417_amd.learned import LearnedFactor
    dev = torch.device("cuda")
    return LearnedFactor(torch.from_numpy(w.row_ptr).to(dev), torch.from_numpy(w.col).to(dev),
                         torch.from_numpy(w.val).to(dev), block_size=bs, theta=theta)


CASES = [("fe27_m3", lambda: W.shifted_fe27(m=3, k=2, seed=3), 3),
         ("fe27_m4", lambda: W.shifted_fe27(m=4, k=2, seed=4), 3),
         ("fe27_m5", lambda: W.shifted_fe27(m=5, k=2, seed=5), 3),
         ("laplace2d_12", lambda: W.shifted_laplace2d(m=12, k=3, seed=7), 1)]
# Norm-wise gradient bound per case.  On the 27-node graph every weight
# gradient is a sum over only 316 edges (27 nodes) with strong cancellation,
# so the BF16 operand rounding of the backward products is averaged over few
# terms and the relative error is larger; the direction (cosine) bound is the
# same for every case.
GRAD_REL = {"fe27_m3": 5e-2}


@pytest.mark.parametrize("name,make,bs", CASES, ids=[c[0] for c in CASES])
def test_forward_C_matches_oracle(name, make, bs):
    w = make()
    theta = perturbed_theta(bs, 11)
    f = factor_for(w, bs, theta)
    g = LR.Graph(w.row_ptr, w.col, w.val, bs)
    assert (f.nodes, f.edges) == (g.N, g.E)
    rp, ci, cv = f.forward()
    torch.cuda.synchronize()
    lp, lc, lv = LR.csr_C(torch.from_numpy(bf16_round(theta).astype(np.float64)), g,
                          w.row_ptr, w.col)
    assert np.array_equal(rp.cpu().numpy(), lp) and np.array_equal(ci.cpu().numpy(), lc)
    got = cv.cpu().numpy()
    err = np.linalg.norm(got - lv) / np.linalg.norm(lv)
    print(name, "C rel err", err)
    assert err <= 1e-2
    assert np.all(np.abs(got - lv) <= 3e-2 * np.abs(lv).max())
    f.close()


@pytest.mark.parametrize("name,make,bs", CASES, ids=[c[0] for c in CASES])
def test_loss_and_gradient_match_oracle(name, make, bs):
    w = make()
    theta = perturbed_theta(bs, 12)
    f = factor_for(w, bs, theta)
    rng = np.random.default_rng(13)
    nb = 4
    Y = rng.standard_normal((w.n, nb)); Z = rng.standard_normal((w.n, nb))
    Yd = torch.from_numpy(Y.astype(np.float32)).cuda().contiguous()
    Zd = torch.from_numpy(Z.astype(np.float32)).cuda().contiguous()
    loss, grad = f.loss_grad(Yd, Zd)
    grad = grad.cpu().numpy().astype(np.float64)
    g = LR.Graph(w.row_ptr, w.col, w.val, bs)
    th = torch.from_numpy(bf16_round(theta).astype(np.float64)).requires_grad_(True)
    # oracle with the pairs the GPU saw (FP32 values)
    L = LR.loss(th, g, Y.astype(np.float32).astype(np.float64),
                Z.astype(np.float32).astype(np.float64))
    L.backward()
    ref = th.grad.numpy()
    print(name, "loss", loss, float(L.detach()))
    cos = float(grad @ ref / (np.linalg.norm(grad) * np.linalg.norm(ref)))
    rel = float(np.linalg.norm(grad - ref) / np.linalg.norm(ref))
    print(name, "grad cosine", cos, "rel", rel)
    # per parameter group: every block sees its gradient (none silently zero)
    off, groups = 0, []
    for pname, shp in LR.param_shapes(bs):
        cnt = int(np.prod(shp))
        gr, rf = grad[off:off + cnt], ref[off:off + cnt]
        nr = np.linalg.norm(rf)
        c = float(gr @ rf / (np.linalg.norm(gr) * nr)) if nr > 0 else 1.0
        groups.append((pname, c, float(np.linalg.norm(gr - rf) / max(nr, 1e-300)),
                       float(nr / np.linalg.norm(ref))))
        off += cnt
    for gname, c, r, share in groups:
        print("  %-7s cos %.6f rel %.3e share %.3e" % (gname, c, r, share))
    assert abs(loss - float(L)) <= 1e-2 * abs(float(L))
    assert cos >= 0.999 and rel <= GRAD_REL.get(name, 2e-2)
    for gname, c, r, share in groups:
        if share > 1e-3:
            assert c >= 0.99, (gname, c)
    f.close()


def test_C_structure_at_size():
    """Lower triangular with a positive diagonal on every row (C C^T SPD)."""
    w = W.shifted_fe27(m=12, k=2, seed=21)
    f = factor_for(w, 3, perturbed_theta(3, 14, scale=0.2))
    rp, ci, cv = f.forward()
    rp, ci, cv = rp.cpu().numpy(), ci.cpu().numpy(), cv.cpu().numpy()
    rows = np.repeat(np.arange(w.n), np.diff(rp))
    assert np.all(ci <= rows)
    d = cv[ci == rows]
    assert d.size == w.n and np.all(d > 0) and np.all(np.isfinite(cv))
    f.close()


def test_learned_C_drives_the_solver():
    """C from the network used as the inner preconditioner: the FP64 outer
    residual reaches the tolerance (the learned part cannot break the
    method: M_cg stays SPD)."""
    from paper_1805_12417_amd import solver as S
    w = W.shifted_fe27(m=6, k=4, seed=22)
    from paper_1805_12417_amd.learned import initial_params
    for prec in (S.PREC_MIXED, S.PREC_FP64):
        s, b = S.from_workload(w, precision=prec)
        f = factor_for(w, 3, initial_params(3, seed=5))
        pc = f.preconditioner(s)
        x, st = s.solve(b, pc, rtol_out=1e-8, rtol_in=1e-4)
        print("precision", prec, st.status_name, st.outer_its, st.inner_its_total,
              st.final_relres)
        assert st.status == 0 and st.final_relres <= 1e-8
        f.close(); s.close()


def test_training_gains_over_jacobi_on_a_held_out_matrix():
    """Train on two FE-like matrices (pairs y = M_mr z, z ~ N(0, I)), then
    precondition the inner CG of a third: fewer iterations than the network's
    starting point and than Jacobi."""
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import learned as LL
    train_w = [W.shifted_fe27(m=10, k=4, seed=300 + i) for i in range(2)]
    ev = W.shifted_fe27(m=10, k=4, seed=310)
    solvers = [S.from_workload(w, precision=S.PREC_FP64)[0] for w in train_w]
    factors = [factor_for(w, 3, LL.initial_params(3, 0)) for w in train_w]
    pairs = [LL.make_pairs(s, 128, "mx", seed=40 + i) for i, s in enumerate(solvers)]
    theta, hist = LL.train(factors, pairs, steps=300, nb=16, lr=3e-3, seed=2)
    assert np.mean(hist[-30:]) < 0.6 * np.mean(hist[:10])
    se, _ = S.from_workload(ev, precision=S.PREC_FP64)

    def its(pc):
        out = []
        for sd in (1, 2):
            g = torch.Generator(device="cuda").manual_seed(sd)
            r = torch.randn(ev.n, dtype=torch.float64, device="cuda", generator=g)
            z, rc, it = se.pcg(r, pc, rtol=1e-6, maxit=20000)
            assert rc == 0
            out.append(it)
        return float(np.mean(out))

    fe = factor_for(ev, 3, LL.initial_params(3, 0))
    it_init = its(fe.preconditioner(se))
    fe.set_params(theta)
    it_trained = its(fe.preconditioner(se))
    it_jacobi = its(se.preconditioner("jacobi"))
    it_ic = its(se.preconditioner("ildl0"))
    # the IC-style ILDL^T(0) is reported next to it: on these matrices it
    # needs fewer iterations than the learned factor (which is cheaper per
    # iteration); the gain asserted is over Jacobi and the untrained network
    print("inner CG iterations: jacobi %.0f, untrained %.0f, trained %.0f, IC-style %.0f" % (
        it_jacobi, it_init, it_trained, it_ic))
    assert it_trained < 0.8 * it_jacobi and it_trained < 0.8 * it_init
    for f in factors + [fe]:
        f.close()


def test_adam_step_matches_kingma_ba():
    """mcg_learned_adam against Adam's update (Kingma & Ba 2015, Algorithm 1)
    written out in FP64 NumPy, over three steps with bias correction."""
    import ctypes as C
    from paper_1805_12417_amd import _native as N
    rng = np.random.default_rng(31)
    P = 1000
    theta = rng.standard_normal(P).astype(np.float32)
    m = np.zeros(P); v = np.zeros(P); th = theta.astype(np.float64)
    dev = torch.device("cuda")
    t_th = torch.from_numpy(theta.copy()).to(dev)
    t_m1 = torch.zeros(P, dtype=torch.float32, device=dev)
    t_m2 = torch.zeros(P, dtype=torch.float32, device=dev)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    # the kernel takes FP32 hyperparameters: the reference uses the same values
    # (1 - fp32(0.999) differs from 1e-3 by 1.3e-5 relative)
    rb1, rb2, rlr, reps = (float(np.float32(v)) for v in (b1, b2, lr, eps))
    for step in (1, 2, 3):
        g = rng.standard_normal(P).astype(np.float32)
        t_g = torch.from_numpy(g).to(dev)
        rc = N.lib().mcg_learned_adam(P, C.c_void_p(t_th.data_ptr()), C.c_void_p(t_g.data_ptr()),
                                      C.c_void_p(t_m1.data_ptr()), C.c_void_p(t_m2.data_ptr()),
                                      lr, b1, b2, eps, step, None)
        assert rc == 0
        m = rb1 * m + (1 - rb1) * g
        v = rb2 * v + (1 - rb2) * g.astype(np.float64) ** 2
        mhat = m / (1 - rb1 ** step)
        vhat = v / (1 - rb2 ** step)
        th = th - rlr * mhat / (np.sqrt(vhat) + reps)
    torch.cuda.synchronize()
    assert np.allclose(t_m1.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
    assert np.allclose(t_m2.cpu().numpy(), v, rtol=1e-5, atol=1e-9)
    assert np.allclose(t_th.cpu().numpy(), th, rtol=0, atol=1e-5 * lr + 1e-6)


def test_solve_record_returns_the_inner_solves():
    """minres_cg_solve_record: the first recorded right-hand side is b - A x0,
    every recorded pair satisfies the inner stopping rule against the
    oracle's M_mr apply (||M_mr z - y|| <= rtol_in ||y||), one pair per inner
    solve, and the solve itself equals the plain solve bitwise."""
    import oracle as O
    from paper_1805_12417_amd import solver as S
    w = W.shifted_fe27(m=6, k=4)
    s, b = S.from_workload(w, precision=S.PREC_FP64)
    pc = s.preconditioner("jacobi")
    x, st, Y, Z = s.solve_record(b, pc, 64, rtol_out=1e-9, rtol_in=1e-5)
    x2, st2 = s.solve(b, pc, rtol_out=1e-9, rtol_in=1e-5)
    assert st.status == 0 and torch.equal(x, x2)
    assert Y.shape[1] == st.outer_its + 1 == Z.shape[1]
    Yh, Zh = Y.cpu().numpy(), Z.cpu().numpy()
    assert np.array_equal(Yh[:, 0], w.b)
    for i in range(Yh.shape[1]):
        r = O.mmr_apply(w.row_ptr, w.col, w.val, w.Vhat, w.lam, Zh[:, i]) - Yh[:, i]
        assert np.linalg.norm(r) <= 1.01e-5 * np.linalg.norm(Yh[:, i]), i
    # a smaller cap keeps the first pairs
    _, _, Y3, Z3 = s.solve_record(b, pc, 3, rtol_out=1e-9, rtol_in=1e-5)
    assert Y3.shape[1] == 3 and torch.equal(Y3, Y[:, :3]) and torch.equal(Z3, Z[:, :3])
