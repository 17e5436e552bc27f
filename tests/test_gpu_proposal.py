"""Learned sketch proposal on the GPU against the FP64 oracle.

Network kernels (FP32) against oracle/convnet.py: forward, backward, capture loss and its
gradient, Adam; small sizes that span several grid tiles and a ragged channel tile
(20 channels = 16 + 4), and the full network (n = 2048, 4 x 64 channels, width 9) on two
states. The projected-residual judge and the observation swap of cycled runs against the
n = 40 oracle problem.

FP32 tolerances: normwise 1e-4 (the FP32 bar); ReLU decisions are taken in each side's
own precision, so at full size a pre-activation within FP32 rounding of zero may switch
sides; the gradient bound there is derived in the test.
"""

import numpy as np
import pytest

from oracle import convnet, fourdvar
from synthetic import net_init
from tests._problems import oracle_problem, rel, riot_for, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(flat, shapes):
    out, o = [], 0
    for cout, cin, width in shapes:
        nw = cout * cin * width
        out.append((flat[o: o + nw].reshape(cout, cin, width), flat[o + nw: o + nw + cout]))
        o += nw + cout
    return out


def _net(n, k, channels, layers, width, batch, seed, segments=1, in_channels=1):
    from paper_1906_01413_amd import ProposalNet
    net = ProposalNet(n, k=k, channels=channels, layers=layers, width=width, batch_max=batch,
                      segments=segments, in_channels=in_channels)
    params = net_init(seed, net.layer_shapes())
    # biases drawn too, so that the bias paths are exercised; both sides see FP32 values
    rng = np.random.default_rng(seed + 1)
    params = [(W.astype(np.float32).astype(np.float64),
               (0.1 * rng.standard_normal(b.size)).astype(np.float32).astype(np.float64))
              for W, b in params]
    net.set_params(_flat(params))
    return net, params


def _states(batch, n, seed, in_channels=1):
    x = 8.0 + 3.0 * np.random.default_rng(seed).standard_normal((batch, in_channels, n))
    return x[:, 0] if in_channels == 1 else x


# 3 grid tiles of 64 points, a ragged channel tile (20 = 16 + 4); without and with the
# localized head (3 segments of 64 points, 2 channels each)
CONFIGS = {
    "plain": dict(n=192, k=5, channels=20, layers=3, width=5, batch=3, segments=1),
    "segmented": dict(n=192, k=6, channels=20, layers=3, width=5, batch=3, segments=3),
    # three input fields per sample, 2 segments, 2 layers of width 3
    "multi_input": dict(n=128, k=4, channels=16, layers=2, width=3, batch=2, segments=2,
                        in_channels=3),
}


@pytest.fixture(scope="module", params=list(CONFIGS))
def small(request):
    cfg = CONFIGS[request.param]
    net, params = _net(**cfg, seed=11)
    return net, params, _states(cfg["batch"], cfg["n"], 12, cfg.get("in_channels", 1)), cfg


def test_forward_matches_oracle(small):
    net, params, X, cfg = small
    N = to_np(net.forward(X))
    for s in range(X.shape[0]):
        ref, _ = convnet.forward(params, X[s], cfg["segments"])
        assert rel(N[s], ref.T) < 1e-5, s


def test_backward_matches_oracle(small):
    net, params, X, cfg = small
    gN = np.random.default_rng(13).standard_normal((X.shape[0], cfg["k"], cfg["n"])).astype(np.float32)
    net.forward(X)
    g = to_np(net.backward(torch.tensor(gN, device="cuda")))
    ref = None
    for s in range(X.shape[0]):
        _, acts = convnet.forward(params, X[s], cfg["segments"])
        gs = convnet.backward(params, acts, gN[s].astype(np.float64).T, cfg["segments"])
        ref = gs if ref is None else [(a + c, b + d) for (a, b), (c, d) in zip(ref, gs)]
    for (gW, gb), (rW, rb) in zip(_unflat(g, net.layer_shapes()), ref):
        assert rel(gW, rW) < 1e-4
        assert rel(gb, rb) < 1e-4


def test_capture_loss_matches_oracle(small):
    net, _, _, cfg = small
    b, k, n = cfg["batch"], cfg["k"], cfg["n"]
    rng = np.random.default_rng(14)
    N = rng.standard_normal((b, k, n)).astype(np.float32)
    V = np.stack([np.linalg.qr(rng.standard_normal((n, k)))[0].T for _ in range(b)])
    w = rng.uniform(0.1, 2.0, (b, k))
    loss, gN = net.capture_loss(torch.tensor(N, device="cuda"), V, w)
    gN = to_np(gN)
    for s in range(b):
        lo, go = convnet.capture_loss(N[s].astype(np.float64).T, V[s].T, w[s])
        assert abs(loss[s] - lo) <= 1e-10 * abs(lo)
        assert rel(gN[s], go.T) < 1e-6  # FP64 result rounded to FP32


def test_adam_matches_oracle(small):
    net, params, _, _ = small
    rng = np.random.default_rng(15)
    p = _flat(params)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr = 1e-3
    net.set_params(p.astype(np.float32))
    q = p.copy()
    for t in (1, 2):
        g = rng.standard_normal(p.size).astype(np.float32).astype(np.float64)
        net.set_params(grads=g.astype(np.float32))
        net.adam(lr)
        q, m, v = convnet.adam(q, g, m, v, t, lr)
    got, _ = net.params()
    assert np.max(np.abs(to_np(got) - q) - (1e-6 * np.abs(q) + 1e-4 * lr)) <= 0
    net.set_params(p.astype(np.float32))


def test_train_step_is_the_composition_and_lowers_the_loss(small):
    net, params, X, cfg = small
    from paper_1906_01413_amd import ProposalNet
    b, k, n, S = cfg["batch"], cfg["k"], cfg["n"], cfg["segments"]
    # targets a network of this shape can reach: the orthonormalised outputs of another
    # ("teacher") network, evaluated by the oracle
    teacher = net_init(99, [(c, ci, wd) for c, ci, wd in net.layer_shapes()])
    V = np.stack([np.linalg.qr(convnet.forward(teacher, X[s], S)[0])[0].T for s in range(b)])
    w = np.random.default_rng(16).uniform(0.5, 2.0, (b, k))
    # the same step by the separate calls on a second network with the same start
    twin = ProposalNet(n, k=k, channels=cfg["channels"], layers=cfg["layers"],
                       width=cfg["width"], batch_max=b, segments=S,
                       in_channels=cfg.get("in_channels", 1))
    twin.set_params(_flat(params).astype(np.float32))
    net.set_params(_flat(params).astype(np.float32))
    l0 = net.train_step(X, V, w, 1e-2)
    N = twin.forward(X)
    l1, gN = twin.capture_loss(N, V, w)
    twin.backward(gN)
    twin.adam(1e-2)
    assert np.array_equal(l0, l1)
    assert torch.equal(net.params()[0], twin.params()[0])
    for _ in range(60):
        last = net.train_step(X, V, w, 1e-2)
    assert np.mean(last) < np.mean(l0) - 0.2, (np.mean(l0), np.mean(last))
    net.set_params(_flat(params).astype(np.float32))


@pytest.mark.parametrize("segments", [1, 16])
def test_full_size_network_matches_oracle(segments):
    """n = 2048, 4 layers x 64 channels, width 9, k = 64, two states."""
    net, params = _net(n=2048, k=64, channels=64, layers=4, width=9, batch=2, seed=21,
                       segments=segments)
    X = _states(2, 2048, 22)
    N = to_np(net.forward(X))
    gN = np.random.default_rng(23).standard_normal((2, 64, 2048)).astype(np.float32)
    g = to_np(net.backward(torch.tensor(gN, device="cuda")))
    ref, near0 = None, 0
    for s in range(2):
        No, acts = convnet.forward(params, X[s], segments)
        assert rel(N[s], No.T) < 1e-5
        for a in acts[1:-1]:
            near0 += int(np.sum((a > 0) & (a < 1e-5 * np.max(np.abs(a)))))
        gs = convnet.backward(params, acts, gN[s].astype(np.float64).T, segments)
        ref = gs if ref is None else [(a + c, b + d) for (a, b), (c, d) in zip(ref, gs)]
    # a hidden unit whose FP32 and FP64 ReLU decisions differ contributes one term of
    # the same size as the others to a few gradient sums. Units within 1e-5 of zero on
    # the positive side (near0), and as many on the negative side, may differ; out of
    # 3 x 64 x 2048 x 2 units they drift the normwise error by about sqrt(2 near0 / units)
    units = 3 * 64 * 2048 * 2
    tol = 1e-4 + 3.0 * np.sqrt(2 * near0 / units)
    for (gW, gb), (rW, rb) in zip(_unflat(g, net.layer_shapes()), ref):
        assert rel(gW, rW) < tol
        assert rel(gb, rb) < tol


def test_proj_residual_matches_oracle():
    """riot_proj_residual on the n = 40 problem: the exact top eigenvectors of A (oracle's
    dense Hessian) are an invariant subspace; a random orthonormal block is not."""
    _, p = oracle_problem("l96_n40", 0)
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    lam, U = np.linalg.eigh(A)
    r = riot_for(p, 40)
    r.linearize(torch.tensor(p.xb, device="cuda"), want_cost=False)
    from paper_1906_01413_amd import colmajor
    Vt = colmajor(U[:, ::-1][:, :12].copy())
    assert r.proj_residual(Vt, r.hess_apply(Vt)) < 1e-10
    Q = np.linalg.qr(np.random.default_rng(24).standard_normal((40, 9)))[0]
    Qt = colmajor(Q)
    got = r.proj_residual(Qt, r.hess_apply(Qt))
    want = fourdvar.proj_residual(Q, A @ Q)
    assert abs(got - want) <= 1e-10 * want


def test_set_obs_equals_a_fresh_handle():
    """New observed values through riot_set_obs give the innovation and gradient of a
    handle created with them (bitwise), and the handle refuses products until linearised."""
    from paper_1906_01413_amd import RiotError
    _, p = oracle_problem("l96_n40", 0)
    r = riot_for(p, 8)
    x = torch.tensor(p.xb, device="cuda")
    y2 = p.y + np.random.default_rng(25).standard_normal(p.y.size)
    r.linearize(x, want_cost=False)
    r.set_obs(y2)
    with pytest.raises(RiotError):
        r.hess_apply(torch.ones(40, dtype=torch.float64, device="cuda"))
    d, g, J = r.linearize(x)
    p.y = y2
    r2 = riot_for(p, 8)
    d2, g2, J2 = r2.linearize(x)
    assert torch.equal(d, d2) and torch.equal(g, g2) and J == J2


def test_learned_proposal_gain_on_cycled_l96():
    """The cycled n = 2048 experiment, shortened: 40 training cycles, 1500 Adam steps of the
    GPU kernels, 12 test cycles (exact increment by CG on 2 of them). The trained network's
    own columns must hold far more of each test cycle's leading eigen-subspace than random
    columns (k / n on average), the sketch built from them must judge no worse than about
    the Gaussian sketch of the same size, and every fallback decision follows the judge."""
    from paper_1906_01413_amd import proposal
    from synthetic import CYCLED, cycled_draws, workload
    cfg = dict(CYCLED)
    w = workload(cfg["workload"])
    s = proposal.run_experiment(w, cycled_draws(0, 52), cfg, net_init(3, proposal.net_shapes(cfg)),
                                train_cycles=40, test_cycles=12, train_steps=1500)
    print(s)
    assert s["train_loss_last"] < s["train_loss_first"] - 0.5
    assert s["net_columns_capture_mean"] > 5.0 * s["random_columns_capture"]
    assert s["rho_ratio_learned_over_gauss_m_median"] < 1.5
    assert 0 <= s["fallbacks"] <= s["cycles"] == 12
