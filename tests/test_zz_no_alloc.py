"""The allocation-free prediction (qw_mlp_predict_static), through the C ABI:
the same means and spreads as qw_mlp_predict on the same network, bit for
bit (the same kernels, only the activations live in the library's static
scratch array instead of the workspace), on two calls in a row, the second
with a smaller batch; batches beyond the static maximum are refused."""
import numpy as np
import pytest

from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def make_net():
    import torch
    s = W.SURROGATE_SHAPE
    shift, scale = W.surrogate_input_map()
    net = qw.MLP(s["n_in"], s["width"], s["depth"], s["n_out"], s["n_nets"], max_batch=1024, shift=shift,
                 scale=scale)
    net.set_params(torch.from_numpy(np.concatenate(
        [W.mlp_init_params(11 + k, s["n_in"], s["width"], s["depth"], s["n_out"]) for k in range(s["n_nets"])])))
    rng = np.random.default_rng(5)
    net.set_output_map(rng.standard_normal(s["n_out"]) * 1e-3, 1e-3 + rng.random(s["n_out"]))
    net.set_spread_weights(1.0 + rng.random(s["n_out"]))
    return net


def queries(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    lo = np.array([r[0] for r in W.SURROGATE_INPUT_RANGES])
    hi = np.array([r[1] for r in W.SURROGATE_INPUT_RANGES])
    return torch.as_tensor(lo + (hi - lo) * rng.random((n, 5)), dtype=torch.float32, device="cuda")


def predict_static(net, x):
    import torch
    B = x.shape[0]
    mean = torch.empty((B, net.shape.n_out), dtype=torch.float32, device="cuda")
    spread = torch.empty(B, dtype=torch.float32, device="cuda")
    qw.qw_mlp_predict_static(net.h, x.data_ptr(), B, mean.data_ptr(), spread.data_ptr(), net.stream())
    return mean, spread


def test_static_prediction_equals_workspace_prediction():
    net = make_net()
    for i, B in enumerate((256, 37)):  # two calls in a row, the second smaller
        print(f"[case] predict_static B={B}", flush=True)
        x = queries(B, seed=i)
        m_ref, s_ref = net.predict(x)
        m, s = predict_static(net, x)
        assert np.array_equal(m.cpu().numpy(), m_ref.cpu().numpy()), B
        assert np.array_equal(s.cpu().numpy(), s_ref.cpu().numpy()), B
    net.close()


def test_static_prediction_refuses_batches_beyond_the_maximum():
    net = make_net()
    x = queries(qw.QW_MLP_STATIC_MAX_BATCH + 1, seed=9)
    with pytest.raises(qw.QWError):
        predict_static(net, x)
    net.close()
