"""GPU parity of the adjoint (backward) kernel against the oracle's
scatter-form transpose, the dot-product identity and autograd checks."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def rand_params(rng, h, w, B):
    return synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), rng.uniform(0, 20),
                             rng.uniform(0.05, 0.4), rng.uniform(0.5, 8.0), B,
                             -int(rng.integers(0, B)), -int(rng.integers(0, B)))


@pytest.mark.parametrize("seed", range(5))
def test_adjoint_matches_oracle_f64(fov, orc, dev, seed):
    rng = np.random.default_rng(200 + seed)
    h, w, c = int(rng.integers(1, 120)), int(rng.integers(1, 150)), int(rng.integers(1, 4))
    B = int(rng.choice([4, 8, 16, 32]))
    p = rand_params(rng, h, w, B)
    g = rng.random((c, h, w))
    got = fov.backward(torch.from_numpy(g).to(dev), p, layout="CHW").cpu().numpy()
    ref = orc.adjoint(g, p)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max()), (h, w, c, p)


def test_adjoint_matches_oracle_f32(fov, orc, dev):
    rng = np.random.default_rng(7)
    h, w = 96, 130
    p = rand_params(rng, h, w, 32)
    g = rng.random((3, h, w)).astype(np.float32)
    got = fov.backward(torch.from_numpy(g).to(dev), p, layout="CHW").cpu().numpy()
    ref = orc.adjoint(g.astype(np.float64), p)
    assert np.max(np.abs(got - ref)) <= 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 5), (2, 2, 2), (1, 9, 1)])
def test_adjoint_degenerate(fov, orc, dev, shape):
    g = np.random.default_rng(1).random(shape)
    p = synth.params_dict(0, 0, 0, 1.0, 6.0, 4)
    got = fov.backward(torch.from_numpy(g).to(dev), p, layout="CHW").cpu().numpy()
    assert np.max(np.abs(got - orc.adjoint(g, p))) <= 1e-12


def test_adjoint_equals_explicit_transpose(fov, orc, dev):
    h, w = 24, 30
    p = synth.params_dict(9.3, 4.1, 2, 0.5, 4.0, 8, -2, -5)
    A = orc.explicit_matrix(h, w, p)
    g = np.random.default_rng(2).random((1, h, w))
    got = fov.backward(torch.from_numpy(g).to(dev), p, layout="CHW").cpu().numpy().reshape(-1)
    assert np.max(np.abs(got - A.T @ g.reshape(-1))) <= 1e-12


def test_dot_product_identity_gpu(fov, dev):
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.random((4, 3, 80, 96))).to(dev)
    y = torch.from_numpy(rng.random((4, 3, 80, 96))).to(dev)
    plist = [rand_params(rng, 80, 96, 16) for _ in range(4)]
    ax = fov.forward(x, plist)
    aty = fov.backward(y, plist)
    lhs, rhs = float((ax * y).sum()), float((x * aty).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradcheck_f64(fov, dev):
    # 3x64x64 float64, e0 = 0 and 16 px fragments so most fragments blur.
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.random((1, 3, 64, 64))).to(dev).requires_grad_(True)
    p = synth.params_dict(20.0, 40.0, 0.0, 0.03, 12.0, 16)
    assert torch.autograd.gradcheck(lambda t: fov.foveate(t, p), (x,), eps=1e-6, atol=1e-9, rtol=1e-7,
                                    fast_mode=True)


def test_autograd_backward_is_adjoint(fov, orc, dev):
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.random((2, 3, 50, 70))).to(dev).requires_grad_(True)
    plist = [rand_params(rng, 50, 70, 16) for _ in range(2)]
    y = fov.foveate(x, plist)
    g = torch.from_numpy(rng.random((2, 3, 50, 70))).to(dev)
    y.backward(g)
    gn = g.cpu().numpy()
    for i in range(2):
        ref = orc.adjoint(gn[i], plist[i])
        assert np.max(np.abs(x.grad[i].cpu().numpy() - ref)) <= 1e-12


def test_cfg5_training_batches(fov, orc, dev):
    # batch 32 of 3x224x224 and batch 4 of 3x512x512 float32, fixation uniform
    # over the frame, slope 0.03, cap 12, e0 32; forward + adjoint.
    rng = np.random.default_rng(6)
    for n, s in ((32, 224), (4, 512)):
        x = synth.uniform_frames((n, 3, s, s), seed=n)
        plist = [synth.params_cfg5(rng, s, s) for _ in range(n)]
        xt = torch.from_numpy(x).to(dev).requires_grad_(True)
        y = fov.foveate(xt, plist)
        g = torch.from_numpy(synth.uniform_frames((n, 3, s, s), seed=n + 1)).to(dev)
        y.backward(g)
        torch.cuda.synchronize()
        yn, gx = y.detach().cpu().numpy(), xt.grad.cpu().numpy()
        for i in (0, n - 1):
            ys, xs = rng.integers(0, s, 400), rng.integers(0, s, 400)
            ref = orc.forward_points(x[i].astype(np.float64), plist[i], ys, xs)
            assert np.max(np.abs(yn[i][:, ys, xs].T - ref)) <= 2e-5
        i = n // 2
        ref = orc.adjoint(g[i].cpu().numpy().astype(np.float64), plist[i])
        assert np.max(np.abs(gx[i] - ref)) <= 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("B", [64, 24])
def test_adjoint_largest_and_odd_blocks_f64(fov, orc, dev, B):
    # 64 px fragments use four output tasks per thread in the vertical gather
    rng = np.random.default_rng(300 + B)
    h, w, c = 150, 170, 2
    p = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 5.0, 0.2, 16.0, B,
                          -int(rng.integers(0, B)), -int(rng.integers(0, B)))
    g = rng.random((c, h, w))
    got = fov.backward(torch.from_numpy(g).to(dev), p, layout="CHW").cpu().numpy()
    ref = orc.adjoint(g, p)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


def test_adjoint_frame_table_big_blocks_f64(fov, orc, dev):
    # more frames than travel in the kernel arguments (the kernels read the uploaded frame table)
    # with 64 px fragments (four values per thread, window rows transposed in runs)
    rng = np.random.default_rng(31)
    n, c, h, w = 17, 2, 70, 90
    ps = [synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 5.0, 0.2, 16.0, 64,
                            -int(rng.integers(0, 64)), -int(rng.integers(0, 64))) for _ in range(n)]
    g = rng.random((n, c, h, w))
    got = fov.backward(torch.from_numpy(g).to(dev), ps).cpu().numpy()
    for i in range(n):
        ref = orc.adjoint(g[i], ps[i])
        assert np.max(np.abs(got[i] - ref)) <= 1e-12 * max(1.0, np.abs(ref).max()), i


def test_adjoint_sigma_map_f64(fov, orc, dev):
    # per-fragment sigma from a map (values below 0, NaN and above the cap included), f64
    rng = np.random.default_rng(14)
    h, w, B = 90, 130, 16
    p = synth.params_dict(0, 0, 0, 0, 9.0, B, -5, -11)
    nby, nbx = orc.grid(h, w, p)
    smap = rng.uniform(-1, 11, size=(nby, nbx)).astype(np.float32)
    smap[0, 0] = np.nan
    pd = dict(p, sigma_map=torch.from_numpy(smap.reshape(-1)).to(dev))
    g = rng.random((2, h, w))
    got = fov.backward(torch.from_numpy(g).to(dev), pd, layout="CHW").cpu().numpy()
    ref = orc.adjoint(g, p, sigma_map=smap.astype(np.float64))
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
