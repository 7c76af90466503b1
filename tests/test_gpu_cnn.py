"""The warm-start network on the GPU against the oracle network, and its use
in the solver.

  - FP32 training kernels: forward, loss and every parameter gradient against
    the FP64 oracle (oracle/cnn.c) on the same seeded parameters and inputs;
    one Adam step against the oracle's.
  - BF16 inference kernels (matrix cores) against the oracle forward, within
    the rounding of bf16 activations.
  - Training pairs from the FMG pass, training, and the warm start: every
    sample still meets the same stopping rule, and the cycles saved by the
    trained network are measured against the plain FMG start.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc, inputs

pytestmark = pytest.mark.gpu

SMALL = dict(sigma2=1.0, corr_len=0.2, n_modes=64, n_levels=3, n0=16)  # 16^2, 32^2, 64^2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def seeded(seed, B, n, scale=0.15):
    rng = np.random.default_rng(seed)
    th = (rng.standard_normal(O.cnn_nparams()) * scale).astype(np.float32)
    x = rng.standard_normal((B, 2, n, n)).astype(np.float32)
    t = rng.standard_normal((B, n, n)).astype(np.float32)
    return th, x, t


@pytest.mark.parametrize("n,B", [(16, 2), (32, 3)])
def test_fp32_forward_and_gradient_match_oracle(n, B):
    th, x, t = seeded(11 + n, B, n)
    log(f"fp32 grad n {n} B {B}")
    with fmgmc.Cnn() as net:
        net.set_params(th)
        y = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
        net.forward(dev(x), y, prec="fp32")
        g = np.zeros(O.cnn_nparams(), np.float32)
        loss = net.grad(dev(x), dev(t), g)
        torch.cuda.synchronize()
    yo = O.cnn_forward(th.astype(np.float64), x)
    Lo, go = O.cnn_loss_grad(th.astype(np.float64), x, t)
    ey = np.abs(y.cpu().numpy() - yo).max() / np.abs(yo).max()
    eg = np.abs(g - go).max() / np.abs(go).max()
    log(f"  y rel {ey:.2e}, loss {loss:.6e} vs {Lo:.6e}, grad rel {eg:.2e}")
    assert ey <= 2e-5
    assert abs(loss - Lo) <= 1e-5 * Lo
    assert eg <= 1e-4
    # every layer's weights and biases, separately
    off = 0
    for ci, co in [(2, 32)] + [(32, 32)] * 4 + [(32, 1)]:
        for size in (co * ci * 9, co):
            sl = slice(off, off + size)
            assert np.abs(g[sl] - go[sl]).max() <= 1e-4 * np.abs(go).max() + 1e-4 * np.abs(go[sl]).max()
            off += size


@pytest.mark.parametrize("n,B", [(16, 2), (64, 1)])
def test_fp32_residual_loss_gradient_matches_oracle(n, B):
    """Residual loss mean((x1 - A y)^2), A the stage operator from K = exp(x0)."""
    th, x, _ = seeded(31 + n, B, n)
    with fmgmc.Cnn() as net:
        net.set_params(th)
        g = np.zeros(O.cnn_nparams(), np.float32)
        loss = net.grad(dev(x), None, g, loss="residual")
        torch.cuda.synchronize()
    Lo, go = O.cnn_residual_loss_grad(th.astype(np.float64), x)
    eg = np.abs(g - go).max() / np.abs(go).max()
    log(f"residual loss n {n}: {loss:.6e} vs {Lo:.6e}, grad rel {eg:.2e}")
    assert abs(loss - Lo) <= 1e-5 * Lo
    assert eg <= 1e-4


def test_adam_step_matches_oracle():
    th, x, t = seeded(5, 2, 16)
    with fmgmc.Cnn() as net:
        net.set_params(th)
        g = np.zeros(O.cnn_nparams(), np.float32)
        net.grad(dev(x), dev(t), g)
        net.adam(1e-3)
        net.grad(dev(x), dev(t), g)   # second step with the gradient at the new point
        net.adam(1e-3)
        got = net.params()
    tho = th.astype(np.float64)
    m = np.zeros_like(tho)
    v = np.zeros_like(tho)
    _, g1 = O.cnn_loss_grad(tho, x, t)
    O.adam(tho, g1, m, v, 1, 1e-3)
    _, g2 = O.cnn_loss_grad(tho, x, t)
    O.adam(tho, g2, m, v, 2, 1e-3)
    # each step moves a parameter by about lr; FP32 gradients of tiny entries may flip
    # the sign of a step, so compare with a bound of 2 lr on a few and 1e-5 on most
    d = np.abs(got - tho)
    log(f"adam: max |diff| {d.max():.2e}, 99.9% quantile {np.quantile(d, 0.999):.2e}")
    assert np.quantile(d, 0.999) <= 1e-5 and d.max() <= 4e-3


@pytest.mark.parametrize("n,B", [(16, 3), (32, 2), (64, 2), (128, 1)])
def test_bf16_inference_matches_oracle(n, B):
    th, x, _ = seeded(21 + n, B, n, 0.1)
    with fmgmc.Cnn() as net:
        net.set_params(th)
        y = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
        net.forward(dev(x), y, prec="bf16")
        yf = torch.zeros_like(y)
        net.forward(dev(x), yf, prec="fp32")
        torch.cuda.synchronize()
    yo = O.cnn_forward(th.astype(np.float64), x)
    e = np.abs(y.cpu().numpy() - yo).max() / np.abs(yo).max()
    ef = np.abs(yf.cpu().numpy() - yo).max() / np.abs(yo).max()
    log(f"bf16 n {n}: rel err {e:.2e} (fp32 {ef:.2e})")
    assert e <= 3e-2 and ef <= 2e-5


def test_save_load_roundtrip(tmp_path):
    th, _, _ = seeded(9, 1, 16)
    with fmgmc.Cnn(seed=1) as a, fmgmc.Cnn(seed=2) as b:
        a.set_params(th)
        a.save(tmp_path / "w.bin")
        assert not np.array_equal(b.params(), th)
        b.load(tmp_path / "w.bin")
        assert np.array_equal(b.params(), th)
    with open(tmp_path / "bad.bin", "wb") as f:
        f.write(b"FMGCNN01" + b"\0" * 16)
    with fmgmc.Cnn() as c, pytest.raises(RuntimeError):
        c.load(tmp_path / "bad.bin")


def test_training_pairs_from_the_fmg_pass():
    """x[0] = log K on the stage grid, x[1] has unit RMS, and the targets are finite."""
    level, S = 2, 6
    n = SMALL["n0"] << level
    xi = inputs.mc_normals(S, SMALL["n_modes"], config=5, level=level, purpose=inputs.PURPOSE_CNN_TRAIN)
    xf = torch.zeros((S, 2, n, n), dtype=torch.float32, device="cuda")
    tf = torch.zeros((S, n, n), dtype=torch.float32, device="cuda")
    xc = torch.zeros((S, 2, n // 2, n // 2), dtype=torch.float32, device="cuda")
    tc = torch.zeros((S, n // 2, n // 2), dtype=torch.float32, device="cuda")
    with fmgmc.Context(**SMALL, solver="fp32_ir") as ctx:
        ctx.make_data(level, dev(xi), xc, tc, xf, tf)
        K = torch.zeros((S, n, n), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(level, dev(xi), K)
        Kc = torch.zeros((S, n // 2, n // 2), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(level - 1, dev(xi), Kc)
    torch.cuda.synchronize()
    np.testing.assert_allclose(xf[:, 0].cpu().numpy(), np.log(np.float32(K.cpu().numpy())), atol=2e-6)
    np.testing.assert_allclose(xc[:, 0].cpu().numpy(), np.log(np.float32(Kc.cpu().numpy())), atol=2e-6)
    for x in (xf, xc):
        rms = np.sqrt((x[:, 1].double() ** 2).mean(dim=(1, 2)).cpu().numpy())
        np.testing.assert_allclose(rms, 1.0, rtol=1e-5)
    for t in (tf, tc):
        assert torch.isfinite(t).all() and t.abs().max() > 0


def test_trained_network_saves_cycles_and_keeps_every_q():
    """Trains on 64^2 / 32^2 pairs, then solves unseen samples with and without the warm start."""
    level = 2
    xi_tr = inputs.mc_normals(1536, SMALL["n_modes"], config=5, level=level, purpose=inputs.PURPOSE_CNN_TRAIN)
    xi_te = dev(inputs.mc_normals(256, SMALL["n_modes"], config=5, level=level, purpose=inputs.PURPOSE_CNN_TEST))
    S = xi_te.shape[0]
    with fmgmc.Context(**SMALL, solver="fp32_ir", max_batch=512) as ctx, fmgmc.Cnn(seed=3) as net:
        hist = ctx.train_cnn(net, level, dev(xi_tr), batch=16, lr=2e-3)
        first, last = hist[:16].mean(), hist[-16:].mean()
        log(f"training: {len(hist)} Adam steps, residual loss {first:.4f} -> {last:.4f}")
        assert last < first
        out = {}
        for name, cnn in (("plain", None), ("warm", net)):
            ctx.set_warm_start(cnn, min_n=32)
            qf = torch.zeros(S, dtype=torch.float64, device="cuda")
            qc = torch.zeros_like(qf)
            cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
            fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
            rc = ctx.solve_level(level, xi_te, qf, qc, cyc, fl)
            torch.cuda.synchronize()
            out[name] = (rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy())
    p, w = out["plain"], out["warm"]
    rejected = (w[4] & fmgmc.FLAG_WARM_REJECTED) != 0
    gain = p[3].mean(axis=0) - w[3].mean(axis=0)
    log(f"cycles plain {p[3].mean(axis=0)}, warm {w[3].mean(axis=0)}, saved {gain}, "
        f"warm start rejected for {rejected.sum()} of {S}")
    assert p[0] == 0 and w[0] == 0
    assert not (w[4] & 3).any()
    assert rejected.mean() < 0.5
    assert gain.sum() > 0
    # both starts end at rel-res <= 1e-10: the QoIs agree to the accuracy of the stopping rule
    assert np.max(np.abs(w[1] - p[1]) / np.abs(p[1])) <= 1e-7
    assert np.max(np.abs(w[2] - p[2]) / np.abs(p[2])) <= 1e-7


@pytest.mark.parametrize("n,B", [(16, 3), (64, 2), (128, 2), (512, 1)])
def test_fused_inference_equals_per_layer(n, B):
    """All six layers in one on-chip pass (row strips of 52 valid columns, several
    strips from 64^2 up) against one launch per layer: the same fragments, tap
    order and bf16 rounding points, so the same bits; and the oracle forward."""
    th, x, _ = seeded(41 + n, B, n, 0.1)
    with fmgmc.Cnn() as net:
        net.set_params(th)
        xd = dev(x)
        y1 = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
        y2 = torch.full_like(y1, float("nan"))
        net.forward(xd, y1, prec="bf16")
        net.forward(xd, y2, prec="bf16_fused")
        torch.cuda.synchronize()
    a, b = y1.cpu().numpy(), y2.cpu().numpy()
    log(f"fused n {n}: max |fused - per-layer| {np.abs(a - b).max():.3e}")
    assert np.array_equal(a, b)
    if n <= 128:
        yo = O.cnn_forward(th.astype(np.float64), x)
        assert np.abs(b - yo).max() / np.abs(yo).max() <= 3e-2
