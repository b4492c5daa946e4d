"""GPU parity of the surrogate network's kernels (qw_mlp_*, qw_gemm_bf16_nt)
through the C ABI, against the FP64 MLP oracle.

Bars (bfloat16 unit roundoff u = 2^-8 relative spacing, FP32 accumulation):
* the product: |C - C_exact| <= 2 K 2^-24 sum_k |a_k b_k| + 1e-30 on bfloat16
  inputs (exact products, FP32 sums of K terms);
* forward pass and gradients against the oracle with the same bfloat16
  rounding points: differences come only from FP32-vs-FP64 sums (relative
  K 2^-24 ~ 1.5e-5 for K = 256) and the rare bfloat16 rounding flips they
  cause (a flip moves one stored value by one spacing, 2^-8 relative, for
  about that fraction 1.5e-5 / 2^-8 ~ 0.4% of the values, with random
  signs); outputs within 5e-4 of max|y|, each gradient block within 1e-3
  relative L2;
* against the plain FP64 oracle (no rounding emulation): gradients within
  2e-2 relative L2 -- the bfloat16 storage itself, a few spacings 2^-8
  spread over four layers;
* Adam: the updated FP32 parameters equal the oracle's Adam step on the
  kernel's own gradients to FP32 rounding (4e-6 relative);
* nets of an ensemble are independent: each net's gradients equal those of a
  one-net ensemble holding its parameters, bit for bit;
* weight gradients over a large batch (split into chunks summed in a fixed
  order): the same 1e-3 bar, the FP32 sums now over K = 2000 terms
  (K 2^-24 ~ 1.2e-4 at worst).
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def print_case(**kw):
    print("[case] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("M_,N_,K_", [(1, 1, 16), (37, 70, 48), (64, 64, 64), (256, 256, 256), (4096, 6, 256),
                                      (6, 256, 4096), (100, 33, 1024)])
def test_gemm_matches_exact_product(M_, N_, K_):
    import torch
    print_case(test="gemm", M=M_, N=N_, K=K_)
    rng = np.random.default_rng(M_ * 7 + N_ * 3 + K_)
    a = torch.from_numpy(rng.standard_normal((M_, K_))).to(torch.bfloat16).cuda()
    b = torch.from_numpy(rng.standard_normal((N_, K_))).to(torch.bfloat16).cuda()
    c = torch.full((M_, N_), float("nan"), dtype=torch.float32, device="cuda")
    qw.qw_gemm_bf16_nt(a.data_ptr(), K_, b.data_ptr(), K_, c.data_ptr(), N_, M_, N_, K_,
                       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    A = a.double().cpu().numpy()
    B = b.double().cpu().numpy()
    exact = A @ B.T
    bound = 2 * K_ * 2.0 ** -24 * (np.abs(A) @ np.abs(B).T) + 1e-30
    err = np.abs(c.double().cpu().numpy() - exact)
    assert np.all(err <= bound), float(np.max(err / bound))


def make_net(n_nets=2, width=128, depth=3, B=300, seed=0):
    import torch
    shift, scale = W.surrogate_input_map()
    n_in, n_out = 5, 6
    net = qw.MLP(n_in, width, depth, n_out, n_nets, max_batch=max(B, 64), shift=shift, scale=scale)
    params = np.stack([W.mlp_init_params(seed + k, n_in, width, depth, n_out) for k in range(n_nets)])
    # non-zero biases so that they matter
    rng = np.random.default_rng(seed + 100)
    for k in range(n_nets):
        layers = M.unflatten(params[k], n_in, width, depth, n_out)
        layers = [(Wt, rng.standard_normal(Wt.shape[0]) * 0.1) for Wt, _ in layers]
        params[k] = M.flatten(layers)
    params = params.astype(np.float32).astype(np.float64)  # what the FP32 master copy holds
    net.set_params(torch.from_numpy(params.reshape(-1)))
    lo = np.array([r[0] for r in W.SURROGATE_INPUT_RANGES])
    hi = np.array([r[1] for r in W.SURROGATE_INPUT_RANGES])
    x = (lo + (hi - lo) * rng.random((B, 5))).astype(np.float32).astype(np.float64)
    t = (rng.random((B, n_out)) * 0.5).astype(np.float32).astype(np.float64)
    return net, params, x, t, shift.astype(np.float32).astype(np.float64), scale.astype(np.float32).astype(np.float64)


def test_forward_matches_oracle():
    """Forward pass against the oracle twice: with the oracle rounding to
    bfloat16 where the kernels store (5e-4 of max |y|: FP32 accumulation
    order only), and against the plain FP64 network.  The second bar,
    5e-3 of max |y|, is 2.5 bfloat16 units (2^-9) of the outputs' scale:
    the CPU oracle's own bfloat16-rounded forward differs from its FP64
    forward by 0.8e-3 to 2.0e-3 of max |y| on these networks."""
    import torch
    print_case(test="mlp_forward")
    net, params, x, t, shift, scale = make_net()
    y = net.forward(torch.from_numpy(x)).double().cpu().numpy()
    for k in range(params.shape[0]):
        layers = M.unflatten(params[k], 5, 128, 3, 6)
        ref, _ = M.forward(layers, x, shift, scale, emulate_bf16=True)
        ref64, _ = M.forward(layers, x, shift, scale, emulate_bf16=False)
        ymax = np.max(np.abs(ref64))
        err = np.max(np.abs(y[k] - ref))
        err64 = np.max(np.abs(y[k] - ref64))
        print(f"  net {k}: max |dy| {err:.2e} vs bf16 oracle, {err64:.2e} vs FP64 oracle (max |y| {ymax:.2e})")
        assert err <= 5e-4 * np.max(np.abs(ref))
        assert err64 <= 5e-3 * ymax
    net.close()


def test_gradients_match_oracle():
    import torch
    print_case(test="mlp_gradients")
    net, params, x, t, shift, scale = make_net()
    g, loss = net.gradients(torch.from_numpy(x), torch.from_numpy(t))
    g = g.double().cpu().numpy()
    loss = loss.double().cpu().numpy()
    for k in range(params.shape[0]):
        layers = M.unflatten(params[k], 5, 128, 3, 6)
        lref, _, gref = M.loss_and_grads(layers, x, t, shift, scale, emulate_bf16=True)
        l64, _, g64 = M.loss_and_grads(layers, x, t, shift, scale, emulate_bf16=False)
        assert abs(loss[k] - lref) <= 1e-3 * lref
        got = M.unflatten(g[k], 5, 128, 3, 6)
        for li, ((gw, gb), (rw, rb), (fw, fb)) in enumerate(zip(got, gref, g64)):
            ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
            eb = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
            e64 = np.linalg.norm(gw - fw) / np.linalg.norm(fw)
            print(f"  net {k} layer {li}: dW rel {ew:.2e}, db rel {eb:.2e}, vs plain FP64 {e64:.2e}")
            assert ew <= 1e-3 and eb <= 1e-3
            assert e64 <= 2e-2
    net.close()


def test_gradients_match_oracle_split_k():
    # a batch of 2000 rows at width 256: the weight-gradient products split
    # the batch into chunks that a second kernel sums in a fixed order
    import torch
    print_case(test="mlp_gradients_split_k", batch=2000, width=256, depth=4)
    net, params, x, t, shift, scale = make_net(n_nets=2, width=256, depth=4, B=2000, seed=3)
    g, loss = net.gradients(torch.from_numpy(x), torch.from_numpy(t))
    g = g.double().cpu().numpy()
    loss = loss.double().cpu().numpy()
    for k in range(params.shape[0]):
        layers = M.unflatten(params[k], 5, 256, 4, 6)
        lref, _, gref = M.loss_and_grads(layers, x, t, shift, scale, emulate_bf16=True)
        assert abs(loss[k] - lref) <= 1e-3 * lref
        got = M.unflatten(g[k], 5, 256, 4, 6)
        for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, gref)):
            ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
            eb = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
            print(f"  net {k} layer {li}: dW rel {ew:.2e}, db rel {eb:.2e}")
            assert ew <= 1e-3 and eb <= 1e-3
    net.close()


def test_nets_are_independent_bitwise():
    import torch
    print_case(test="mlp_independent")
    net, params, x, t, shift, scale = make_net(n_nets=3)
    g, _ = net.gradients(torch.from_numpy(x), torch.from_numpy(t))
    for k in range(3):
        one = qw.MLP(5, 128, 3, 6, 1, max_batch=300, shift=shift, scale=scale)
        one.set_params(torch.from_numpy(params[k]))
        g1, _ = one.gradients(torch.from_numpy(x), torch.from_numpy(t))
        assert torch.equal(g1[0], g[k])
        one.close()
    net.close()


def test_adam_step_matches_oracle_on_kernel_gradients():
    import torch
    print_case(test="mlp_adam")
    net, params, x, t, shift, scale = make_net()
    xd, td = torch.from_numpy(x).float().cuda(), torch.from_numpy(t).float().cuda()
    p, m, v = params.copy(), np.zeros_like(params), np.zeros_like(params)
    lr = 3e-3
    for step in (1, 2, 3):
        g, _ = net.gradients(xd, td)
        g = g.double().cpu().numpy()
        net.train_step(xd, td, lr)
        got = net.params().double().cpu().numpy()
        for k in range(p.shape[0]):
            p[k], m[k], v[k] = M.adam_step(p[k], g[k], m[k], v[k], step, lr)
        err = np.max(np.abs(got - p) / (np.abs(p) + lr))
        print(f"  step {step}: max rel param error {err:.2e}")
        assert err <= 4e-6
        p = got.copy()
    net.close()


def test_predict_is_the_ensemble_mean_and_spread():
    import torch
    print_case(test="mlp_predict")
    net, params, x, t, shift, scale = make_net(n_nets=4)
    y = net.forward(torch.from_numpy(x)).double().cpu().numpy()
    osh = np.array([0.5, -1.0, 2.0, 0.0, 1e-3, 3.0], dtype=np.float32).astype(np.float64)
    osc = np.array([2.0, 0.5, 1e-4, 1.0, 3.0, 0.25], dtype=np.float32).astype(np.float64)
    net.set_output_map(osh, osc)
    y = y * osc + osh
    mean, spread = net.predict(torch.from_numpy(x))
    mean, spread = mean.double().cpu().numpy(), spread.double().cpu().numpy()
    assert np.max(np.abs(mean - y.mean(axis=0))) <= 1e-6 * np.max(np.abs(y))
    assert np.max(np.abs(spread - y.std(axis=0, ddof=1).max(axis=1))) <= 1e-5 * np.max(np.abs(y))
    net.close()


def test_training_reduces_the_loss_on_a_smooth_target():
    import torch
    print_case(test="mlp_train")
    shift, scale = W.surrogate_input_map()
    net = qw.MLP(5, 256, 4, 6, 4, max_batch=1024, shift=shift, scale=scale)
    net.set_params(torch.from_numpy(np.concatenate([W.mlp_init_params(k, 5, 256, 4, 6) for k in range(4)])))
    rng = np.random.default_rng(1)
    lo = np.array([r[0] for r in W.SURROGATE_INPUT_RANGES])
    hi = np.array([r[1] for r in W.SURROGATE_INPUT_RANGES])
    u = rng.random((4096, 5))
    x = lo + (hi - lo) * u
    z = 2 * u - 1
    t = np.stack([np.sin(2 * z[:, 0]) * z[:, 1], z[:, 2] ** 2, np.cos(3 * z[:, 3]), z[:, 4] * z[:, 0],
                  np.exp(-z[:, 1] ** 2), 0.1 * z[:, 2]], axis=1) * 0.5
    xd, td = torch.from_numpy(x).float().cuda(), torch.from_numpy(t).float().cuda()
    loss = torch.empty(4, device="cuda")
    _, l0 = net.gradients(xd[:1024], td[:1024])
    l0 = l0.cpu().numpy()
    for it in range(600):
        i = (it % 4) * 1024
        net.train_step(xd[i:i + 1024], td[i:i + 1024], 2e-3, loss)
    _, l1 = net.gradients(xd[:1024], td[:1024])
    l1 = l1.cpu().numpy()
    print(f"  loss {l0} -> {l1}")
    assert np.all(l1 <= 0.05 * l0)
    net.close()
