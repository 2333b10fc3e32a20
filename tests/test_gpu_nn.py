"""GPU parity of the warm-start network kernels against the FP64 oracle
(oracle/nn.py), and the warm start inside the solver on a small ring.

Tolerances: the kernels compute in FP32 (products on the FP32 matrix cores,
FP32 accumulation over at most a few hundred terms), so outputs and
gradients are compared at 1e-4 relative to their largest magnitude.
"""
import numpy as np
import pytest

from oracle import nn as onn
from workloads import configs

pytestmark = pytest.mark.gpu

ARCH = (37, 70, 2, 3, 45)  # ragged: no size is a multiple of the 64-wide tiles
N_ROWS = 130


def _setup(seed=0, n=N_ROWS, arch=ARCH):
    from paper_2501_04340_amd import NN
    rng = np.random.default_rng(seed)
    d = onn.dims(*arch)
    npar = sum(b * (a + 1) for a, b in zip(d[:-1], d[1:]))
    theta = (rng.standard_normal(npar) * 0.3).astype(np.float32)
    X = rng.standard_normal((n, arch[0])).astype(np.float32)
    Cc = rng.uniform(0.5, 1.5, size=(n, arch[3])).astype(np.float32)
    T = rng.standard_normal((n, arch[4])).astype(np.float32)
    net = NN(*arch)
    assert net.n_params == npar
    net.set_params(theta)
    return net, theta, X, Cc, T


def test_forward_matches_oracle(ietilib):
    net, theta, X, Cc, T = _setup()
    pred = net.predict(X, Cc)
    _, _, ref = onn.forward(ARCH, theta.astype(np.float64), X.astype(np.float64), Cc.astype(np.float64))
    assert np.abs(pred - ref).max() <= 1e-4 * np.abs(ref).max()
    assert np.array_equal(net.params(), theta)


def test_loss_and_gradient_match_oracle(ietilib):
    net, theta, X, Cc, T = _setup(1)
    net.set_data(X, Cc, T)
    loss, g = net.loss_grad()
    th = theta.astype(np.float64)
    args = (X.astype(np.float64), Cc.astype(np.float64), T.astype(np.float64))
    ref_loss = onn.loss(ARCH, th, *args)
    ref_g = onn.grad(ARCH, th, *args)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert np.abs(g - ref_g).max() <= 1e-4 * np.abs(ref_g).max()
    # a sub-range of rows
    loss2, g2 = net.loss_grad(17, 50)
    ref2 = onn.grad(ARCH, th, *(a[17:67] for a in args))
    assert np.abs(g2 - ref2).max() <= 1e-4 * np.abs(ref2).max()


def test_one_full_batch_adam_step_matches_oracle(ietilib):
    net, theta, X, Cc, T = _setup(2)
    net.set_data(X, Cc, T)
    th = theta.astype(np.float64)
    args = (X.astype(np.float64), Cc.astype(np.float64), T.astype(np.float64))
    g = onn.grad(ARCH, th, *args)
    lr = 1e-3
    ref, _, _ = onn.adam_step(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr)
    losses = net.train(1, lr, batch=N_ROWS, seed=5)
    new = net.params().astype(np.float64)
    # Adam's first step is lr * g / (|g| + eps): compare where g is not at rounding level
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.abs(new - ref)[big].max() <= 1e-3 * lr + 1e-7
    assert np.all(np.abs(new - th) <= lr * (1 + 1e-3) + 1e-7)
    assert abs(losses[0] - onn.loss(ARCH, th, *args)) <= 1e-5 * losses[0]


def test_training_fits_a_teacher_network(ietilib):
    arch = (12, 64, 2, 2, 20)
    teacher, th_t, X, Cc, _ = _setup(3, n=2048, arch=arch)
    Y = teacher.predict(X, Cc)
    student, _, _, _, _ = _setup(4, n=8, arch=arch)
    student.set_data(X, Cc, Y)
    l0, _ = student.loss_grad()
    losses = student.train(60, 3e-3, batch=128, seed=1)
    l1, _ = student.loss_grad()
    print(f"[gpu-nn] teacher fit: loss {l0:.3e} -> {l1:.3e}")
    assert np.all(np.isfinite(losses)) and l1 <= 0.05 * l0


RING = dict(degree=2, n_el=2, n_theta=12)


@pytest.fixture(scope="module")
def ring(ietilib):
    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.warmstart import RingWarmStart
    prob = configs.ring576(**RING)
    S = Solver(prob)
    W = RingWarmStart(S, prob, window=2, hidden=64, layers=2)
    draws = []
    for i in range(72):
        nu, cur = configs.ring_coefficients(configs.ring_sample_seed(i), n_theta=RING["n_theta"])
        draws.append((nu, configs.ring_load_scale(cur, n_theta=RING["n_theta"])))
    import tempfile
    ds = tempfile.mkdtemp(prefix="ring_ds_")
    X, Cc, T, _ = W.generate(draws[:64], rtol=1e-11, dataset=f"{ds}/rows.bin")
    losses = W.fit(X, Cc, T, epochs=150, lr=2e-3, batch=64, seed=0)
    W.dataset = f"{ds}/rows.bin"
    print(f"[gpu-nn] ring fit: loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    W.attach()
    return prob, S, W, draws[64:]


def test_warm_start_saves_iterations_on_held_out_draws(ring):
    prob, S, W, held = ring
    cold_it, warm_it = [], []
    for nu, scale in held:
        S.set_coefficients(nu, scale)
        S.factor()
        a_c, st_c = S.solve(rtol=1e-8)
        lam_c = S.lambda_()
        a_w, st_w = S.solve(rtol=1e-8, warm_start=True)
        assert st_w["warm_start"] == 1 and st_w["rel_residual0"] < 1.0
        assert st_c["status"] == 0 and st_w["status"] == 0 and st_w["rel_residual"] <= 1e-8
        # the prediction the solver used is the network's
        pred = W.predict_lambda()
        r0 = np.linalg.norm(S.rhs() - S.apply_F(pred)) / np.linalg.norm(S.rhs())
        assert abs(r0 - st_w["rel_residual0"]) <= 1e-3 * r0
        assert np.abs(a_w - a_c).max() <= 1e-5 * np.abs(a_c).max()
        cold_it.append(st_c["iters"])
        warm_it.append(st_w["iters"])
    print(f"[gpu-nn] held-out: cold iters {np.mean(cold_it):.1f}, warm iters {np.mean(warm_it):.1f}")
    assert np.mean(warm_it) < np.mean(cold_it)


def test_bad_prediction_falls_back_to_zero(ring):
    prob, S, W, held = ring
    nu, scale = held[0]
    S.set_coefficients(nu, scale)
    S.factor()
    a_c, st_c = S.solve(rtol=1e-8)
    sh, sc, keep = W.net.normalisation()
    W.net.set_normalisation(sh, sc, 1e8 * keep)
    W.attach()
    try:
        a_w, st_w = S.solve(rtol=1e-8, warm_start=True)
    finally:
        W.net.set_normalisation(sh, sc, keep)
        W.attach()
    assert st_w["warm_start"] == -1 and st_w["rel_residual0"] == 1.0
    assert st_w["iters"] == st_c["iters"] and np.array_equal(a_w, a_c)


def test_warm_start_with_mixed_precision(ring):
    from paper_2501_04340_amd.ietidp import PREC_FP64, PREC_MIXED
    prob, S, W, held = ring
    nu, scale = held[1]
    S.set_coefficients(nu, scale)
    S.factor(precision=PREC_MIXED)
    try:
        a_w, st_w = S.solve(rtol=1e-8, warm_start=True)
        a_c, st_c = S.solve(rtol=1e-8)
    finally:
        S.factor(precision=PREC_FP64)
    assert st_w["warm_start"] == 1 and st_w["status"] == 0 and st_w["rel_residual"] <= 1e-8
    assert np.abs(a_w - a_c).max() <= 1e-5 * np.abs(a_c).max()


def test_layout_mismatch_is_rejected(ring):
    from paper_2501_04340_amd import NN
    prob, S, W, held = ring
    other = NN(W.n_feat + 1, 8, 1, W.n_comb, W.n_out)
    with pytest.raises(Exception, match="INVALID_ARG"):
        S.set_warm_start(other, W.feat_patch, W.comb_patch, W.out_row, W.out_sign)


def test_network_file_round_trip(ietilib, tmp_path):
    """ieti_nn_save / ieti_nn_load: the loaded network has the same
    architecture and parameters bit for bit, and predicts the same values."""
    from paper_2501_04340_amd import NN
    net, theta, X, Cc, T = _setup(seed=5)
    path = tmp_path / "net.bin"
    net.save(path)
    back = NN.load(path)
    assert back.arch == net.arch and back.n_params == net.n_params
    assert np.array_equal(back.params(), net.params())
    assert np.array_equal(back.predict(X, Cc), net.predict(X, Cc))


def test_saved_warm_start_drives_the_solver_identically(ring, tmp_path):
    """A ring warm start written to files and loaded into a fresh layout
    gives the same initial multipliers, and the solver the same result."""
    from paper_2501_04340_amd.warmstart import RingWarmStart
    prob, S, W, held = ring
    nu, scale = held[2]
    W.save(tmp_path / "ring")
    W2 = RingWarmStart.load(S, prob, tmp_path / "ring")
    S.set_coefficients(nu, scale)
    S.factor()
    p1 = W.predict_lambda()
    a1, st1 = S.solve(rtol=1e-8, warm_start=True)
    W2.attach()
    try:
        p2 = W2.predict_lambda()
        a2, st2 = S.solve(rtol=1e-8, warm_start=True)
        # the handle-level load of the same file
        S.warm_load(tmp_path / "ring.net", *W.layout())
        a3, st3 = S.solve(rtol=1e-8, warm_start=True)
    finally:
        W.attach()
    assert np.array_equal(p1, p2)
    assert st1["iters"] == st3["iters"] and np.array_equal(a1, a3)
    assert st1["iters"] == st2["iters"] and np.array_equal(a1, a2)


def test_normalisation_is_applied_to_inputs_and_outputs(ietilib):
    """With a normalisation the network computes on (x - shift) * scale and
    predicts out_scale times its output; training data are raw rows and the
    loss is taken in the normalised coordinates."""
    net, theta, X, Cc, T = _setup(seed=6)
    rng = np.random.default_rng(6)
    sh = rng.standard_normal(ARCH[0]).astype(np.float32)
    sc = rng.uniform(0.5, 2.0, ARCH[0]).astype(np.float32)
    net.set_normalisation(sh, sc, 3.5)
    Xn = ((X - sh) * sc).astype(np.float64)
    _, _, ref = onn.forward(ARCH, theta.astype(np.float64), Xn, Cc.astype(np.float64))
    pred = net.predict(X, Cc)
    assert np.abs(pred - 3.5 * ref).max() <= 1e-4 * np.abs(3.5 * ref).max()
    net.set_data(X, Cc, T)
    loss, _ = net.loss_grad()
    ref_loss = onn.loss(ARCH, theta.astype(np.float64), Xn, Cc.astype(np.float64), T.astype(np.float64) / 3.5)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    # fitted normalisation: column means and inverse standard deviations, output RMS
    net.fit_normalisation(X, T)
    sh2, sc2, o2 = net.normalisation()
    np.testing.assert_allclose(sh2, X.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(sc2, 1.0 / X.astype(np.float64).std(axis=0), rtol=1e-5)
    assert abs(o2 - np.sqrt(np.mean(T.astype(np.float64) ** 2))) <= 1e-6 * o2


def test_seeded_initial_parameters(ietilib):
    """Glorot-uniform weights (within +-sqrt(6 / (d_in + d_out)) per layer,
    spread over that range), zero biases, identical for the same seed."""
    from paper_2501_04340_amd import NN
    a, b = NN(*ARCH), NN(*ARCH)
    a.init_params(11)
    b.init_params(11)
    pa = a.params()
    assert np.array_equal(pa, b.params())
    b.init_params(12)
    assert not np.array_equal(pa, b.params())
    off = 0
    d = onn.dims(*ARCH)
    for din, dout in zip(d[:-1], d[1:]):
        Wb = pa[off:off + dout * (din + 1)].reshape(dout, din + 1)
        lim = np.sqrt(6.0 / (din + dout))
        assert np.all(Wb[:, din] == 0.0)
        assert np.abs(Wb[:, :din]).max() <= lim * (1 + 1e-6)
        assert np.abs(Wb[:, :din]).max() >= 0.9 * lim and abs(Wb[:, :din].mean()) <= 0.1 * lim
        off += dout * (din + 1)


def test_dataset_file_training_matches_in_memory_training(ring, tmp_path):
    """The solver-written dataset file holds the same rows as the in-memory
    data, and ieti_nn_train_file (seeded init, fitted normalisation, Adam)
    gives bitwise the network of the same steps in memory."""
    from paper_2501_04340_amd.warmstart import RingWarmStart
    prob, S, W, held = ring
    W2 = RingWarmStart(S, prob, window=2, hidden=16, layers=1)
    model = tmp_path / "from_file.net"
    l_file = W2.fit_file(W.dataset, model, epochs=3, lr=2e-3, batch=64, seed=4)
    net_file = W2.net
    rows = np.fromfile(W.dataset, dtype=np.float32, offset=20).reshape(-1, W.n_feat + W.n_comb + W.n_out)
    X, Cc, T = np.split(rows, [W.n_feat, W.n_feat + W.n_comb], axis=1)
    l_mem = W2.fit(X, Cc, T, epochs=3, lr=2e-3, batch=64, seed=4)
    assert np.array_equal(net_file.params(), W2.net.params())
    assert np.allclose(l_file, l_mem, rtol=0, atol=0)
    assert [np.array_equal(u, v) for u, v in zip(net_file.normalisation(), W2.net.normalisation())] == [True] * 3
