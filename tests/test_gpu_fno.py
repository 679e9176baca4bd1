"""GPU surrogate kernels against the FP64 oracle network: forward outputs,
loss and every gradient on the same (BF16-rounded) weights, and short
training runs (plain, and through the cube-symmetry maps) that lower the
loss."""
import numpy as np
import pytest

from oracle import fno as ofno
from gpu_util import say

pytestmark = pytest.mark.gpu


def flat_to_dict(flat, cin, W, m, L):
    K = (2 * m) * (2 * m) * m
    d, o = {}, 0

    def take(n):
        nonlocal o
        v = flat[o:o + n].astype(np.float64)
        o += n
        return v
    d["P"] = take(W * cin).reshape(W, cin)
    d["p"] = take(W)
    d["Q"] = take(W)
    d["q0"] = take(1)
    for l in range(L):
        r = take(K * W * W * 2).reshape(K, W, W, 2)
        d[f"R{l}"] = r[..., 0] + 1j * r[..., 1]
        d[f"W{l}"] = take(W * W).reshape(W, W)
        d[f"b{l}"] = take(W)
    assert o == flat.size
    return d


def dict_to_flat(d, L):
    parts = [d["P"].ravel(), d["p"], d["Q"], d["q0"]]
    for l in range(L):
        R = d[f"R{l}"]
        parts += [np.stack([R.real, R.imag], axis=-1).ravel(), d[f"W{l}"].ravel(), d[f"b{l}"]]
    return np.concatenate(parts)


@pytest.mark.parametrize("n,cin,W,m,L,B,bf16", [(16, 3, 4, 2, 2, 2, False), (16, 3, 32, 8, 4, 2, True),
                                                (32, 3, 8, 4, 3, 1, True)])
def test_forward_and_gradients_match_oracle(n, cin, W, m, L, B, bf16):
    import torch
    from paper_2205_06690_amd import bse
    rng = np.random.default_rng(3)
    net = bse.Fno(n, cin=cin, width=W, modes=m, layers=L, max_batch=B, bf16_weights=bf16, seed=5)
    p = net.get_params()
    p = p + 0.05 * rng.standard_normal(p.size).astype(np.float32)   # biases non-zero too
    net.set_params(p)
    pc = net.get_params(compute=True)                                 # the weights the kernels use
    x = rng.standard_normal((B, cin, n, n, n)).astype(np.float32)
    t = rng.standard_normal((B, n, n, n)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    yd = torch.empty((B, n, n, n), dtype=torch.float32, device="cuda")
    net.forward(B, xd.data_ptr(), yd.data_ptr())
    d = flat_to_dict(pc, cin, W, m, L)
    y_o, _ = ofno.forward(d, x.astype(np.float64), n, m, L)
    ey = np.abs(yd.cpu().numpy() - y_o).max() / np.abs(y_o).max()
    loss, g = net.loss_grad(B, xd.data_ptr(), td.data_ptr())
    loss_o, g_o = ofno.loss_and_grad(d, x.astype(np.float64), t.astype(np.float64), n, m, L)
    gf = dict_to_flat(g_o, L)
    eg = np.linalg.norm(g - gf) / np.linalg.norm(gf)
    say(f"fno n={n} W={W} m={m} L={L}: rel|dy| {ey:.2e}  loss {loss:.6f} vs {loss_o:.6f}  rel|dgrad| {eg:.2e}")
    assert ey < 1e-4
    assert abs(loss - loss_o) < 1e-5 * abs(loss_o)
    assert eg < 1e-4
    # every parameter family separately
    gd = flat_to_dict(g, cin, W, m, L)
    for k in g_o:
        nrm = np.linalg.norm(g_o[k])
        if nrm > 0:
            assert np.linalg.norm(gd[k] - g_o[k]) / nrm < 1e-3, k


def test_training_lowers_loss():
    import torch
    from paper_2205_06690_amd import bse
    n, B = 16, 4
    rng = np.random.default_rng(0)
    net = bse.Fno(n, cin=3, width=16, modes=4, layers=4, max_batch=B, seed=1)
    x = torch.from_numpy(rng.standard_normal((B, 3, n, n, n)).astype(np.float32)).cuda()
    # a smooth target: a fixed linear map of the first channel
    k = np.fft.fftfreq(n) * n
    filt = 1.0 / (1.0 + k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    t = np.real(np.fft.ifftn(np.fft.fftn(x[:, 0].cpu().numpy(), axes=(1, 2, 3)) * filt, axes=(1, 2, 3)))
    t = torch.from_numpy((-0.5 * t).astype(np.float32)).cuda()
    losses = [net.train_step(B, x.data_ptr(), t.data_ptr(), 3e-3) for _ in range(60)]
    say("training losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]


def test_augmented_training_runs_and_learns():
    """surrogate.train with the cube-symmetry maps on flattened samples: the
    target here (a radial filter of the first channel) commutes with every
    map, so the mapped batches stay consistent and the loss falls."""
    import torch
    from paper_2205_06690_amd import bse, surrogate
    n, N, B = 16, 8, 4
    rng = np.random.default_rng(2)
    net = bse.Fno(n, cin=3, width=16, modes=4, layers=4, max_batch=B, seed=1)
    xs = rng.standard_normal((N, 3, n, n, n))
    k = np.fft.fftfreq(n) * n
    filt = 1.0 / (1.0 + k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    ts = -0.5 * np.real(np.fft.ifftn(np.fft.fftn(xs[:, 0], axes=(1, 2, 3)) * filt, axes=(1, 2, 3)))
    x = torch.from_numpy(xs.reshape(N, 3, -1).astype(np.float32)).cuda()
    t = torch.from_numpy(ts.reshape(N, -1).astype(np.float32)).cuda()
    hist = surrogate.train(net, x, t, epochs=30, batch=B, lr=3e-3, lr_end=3e-4, log=lambda *a: None,
                           augment=True)
    say("augmented training losses", hist[0], hist[-1])
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.5 * hist[0]


def test_adam_updates_match_oracle():
    """Three training steps of the GPU network against the oracle's Adam on
    the same gradients: each step's gradient is read with loss_grad at the
    current weights, the oracle advances FP64 copies of the master weights
    and moments with it, and the GPU's train_step (same batch, so the same
    gradient) must move the master weights the same way.  Steps 2 and 3
    exercise both bias corrections and tell beta1 from beta2."""
    import torch
    from paper_2205_06690_amd import bse
    n, B, lr = 16, 2, 1e-2
    rng = np.random.default_rng(11)
    net = bse.Fno(n, cin=3, width=8, modes=4, layers=2, max_batch=B, bf16_weights=False, seed=3)
    x = torch.from_numpy(rng.standard_normal((B, 3, n, n, n)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((B, n, n, n)).astype(np.float32)).cuda()
    p_orc = {"w": net.get_params().astype(np.float64)}
    st = {}
    for k in range(3):
        p_before = net.get_params().astype(np.float64)
        _, g = net.loss_grad(B, x.data_ptr(), t.data_ptr())
        net.train_step(B, x.data_ptr(), t.data_ptr(), lr)
        p_after = net.get_params().astype(np.float64)
        ofno.adam_step(p_orc, {"w": g.astype(np.float64)}, st, lr=lr)
        d_gpu = p_after - p_before
        d_orc = p_orc["w"] - p_before
        e = np.linalg.norm(d_gpu - d_orc) / np.linalg.norm(d_orc)
        say(f"adam step {k + 1}: rel|d update| {e:.2e}, |update| {np.linalg.norm(d_orc):.3e}")
        assert e < 1e-3, (k, e)
        p_orc["w"] = p_after.copy()        # the next step starts from the GPU's weights


@pytest.mark.parametrize("W,m,B", [(32, 8, 8), (16, 4, 3), (8, 4, 17)])
def test_matrix_core_mix_equals_vector_path(W, m, B):
    """The per-mode channel mix on the matrix cores against the vector-FMA
    path on the same weights and inputs: forward output and every gradient
    agree to FP32 rounding (widths 8, 16 and 32, a batch above 16)."""
    import torch
    from paper_2205_06690_amd import bse
    n, L = 16, 2
    rng = np.random.default_rng(7)
    net = bse.Fno(n, cin=3, width=W, modes=m, layers=L, max_batch=B, bf16_weights=True, seed=2)
    p = net.get_params()
    net.set_params(p + 0.05 * rng.standard_normal(p.size).astype(np.float32))
    x = torch.from_numpy(rng.standard_normal((B, 3, n, n, n)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((B, n, n, n)).astype(np.float32)).cuda()
    out = []
    for path in (0, 1):
        net.set_mix_path(path)
        y = torch.empty((B, n, n, n), dtype=torch.float32, device="cuda")
        net.forward(B, x.data_ptr(), y.data_ptr())
        loss, g = net.loss_grad(B, x.data_ptr(), t.data_ptr())
        out.append((y.cpu().numpy(), loss, g))
    (y0, l0, g0), (y1, l1, g1) = out
    ey = np.abs(y0 - y1).max() / np.abs(y1).max()
    eg = np.linalg.norm(g0 - g1) / np.linalg.norm(g1)
    say(f"mix paths W={W} m={m} B={B}: rel|dy| {ey:.2e}, rel|dgrad| {eg:.2e}")
    assert ey < 1e-5 and eg < 1e-5 and abs(l0 - l1) < 1e-6 * abs(l1)


def test_gather_under_cube_symmetries():
    """The library's batch gather equals index_select, permute and flip of
    the samples for symmetries of the cube (pure copies: bit for bit), and
    rejects bad arguments."""
    import torch
    from paper_2205_06690_amd import bse
    n, cin, B, n_src = 16, 3, 4, 7
    net = bse.Fno(n, cin=cin, width=8, modes=4, layers=1, max_batch=B, seed=2)
    g = torch.Generator().manual_seed(4)
    x = torch.randn((n_src, cin, n ** 3), generator=g).cuda()
    t = torch.randn((n_src, n ** 3), generator=g).cuda()
    xd = torch.empty((B, cin, n ** 3), device="cuda")
    td = torch.empty((B, n ** 3), device="cuda")
    idx = [5, 0, 6, 2]
    sel = torch.tensor(idx, device="cuda")
    for perm, fm in [((0, 1, 2), 0), ((2, 0, 1), 5), ((1, 0, 2), 2), ((2, 1, 0), 7), ((0, 2, 1), 1)]:
        net.gather(idx, n_src, x.data_ptr(), t.data_ptr(), perm, fm, xd.data_ptr(), td.data_ptr())
        flips = [a for a in range(3) if (fm >> a) & 1]
        xr = x.index_select(0, sel).reshape(B, cin, n, n, n).permute(0, 1, *(2 + a for a in perm))
        tr = t.index_select(0, sel).reshape(B, n, n, n).permute(0, *(1 + a for a in perm))
        if flips:
            xr = xr.flip([2 + a for a in flips])
            tr = tr.flip([1 + a for a in flips])
        assert torch.equal(xd, xr.reshape(B, cin, -1)) and torch.equal(td, tr.reshape(B, -1)), (perm, fm)
    say("gather: 5 symmetries equal to permute/flip")
    for bad in [dict(idx=[0, 7, 1, 2]), dict(perm=(0, 0, 1)), dict(fm=8)]:
        with pytest.raises(bse.BseError) as e:
            net.gather(bad.get("idx", idx), n_src, x.data_ptr(), t.data_ptr(), bad.get("perm", (0, 1, 2)),
                       bad.get("fm", 0), xd.data_ptr(), td.data_ptr())
        assert e.value.code == bse.BSE_ERR_ARG
    net.close()
