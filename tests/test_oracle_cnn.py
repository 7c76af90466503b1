"""Pins of the oracle network (oracle/cnn.c): finite differences, an
independent library implementation (torch CPU FP64 conv2d with autograd),
special cases with closed forms, and the closed form of Adam's first step."""
import numpy as np
import pytest

from oracle import oracle as O


def rand_net(rng, cin, F, R, scale=0.3):
    return rng.standard_normal(O.cnn_nparams(cin, F, R)) * scale


def test_parameter_count():
    # 2 -> 32, four 32 -> 32, 32 -> 1, 3x3 kernels with biases
    assert O.cnn_nparams() == 32 * 2 * 9 + 32 + 4 * (32 * 32 * 9 + 32) + 32 * 9 + 1 == 37889


@pytest.mark.parametrize("cin,F,R,n,B", [(2, 4, 2, 6, 2), (1, 3, 1, 5, 1)])
def test_gradient_matches_central_differences(cin, F, R, n, B):
    rng = np.random.default_rng(3)
    th = rand_net(rng, cin, F, R)
    x = rng.standard_normal((B, cin, n, n))
    t = rng.standard_normal((B, n, n))
    L, g = O.cnn_loss_grad(th, x, t, cin, F, R)
    h = 1e-6
    for k in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (O.cnn_loss_grad(tp, x, t, cin, F, R)[0] - O.cnn_loss_grad(tm, x, t, cin, F, R)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_full_size_network_against_torch_autograd():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as Fn
    cin, F, R, n, B = O.CNN_CIN, O.CNN_WIDTH, O.CNN_RES, 7, 2
    rng = np.random.default_rng(5)
    th = rand_net(rng, cin, F, R, 0.1)
    x = rng.standard_normal((B, cin, n, n))
    t = rng.standard_normal((B, n, n))
    y_o, z_o, h_o = O.cnn_forward(th, x, cin, F, R, acts=True)
    L_o, g_o = O.cnn_loss_grad(th, x, t, cin, F, R)
    tt = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    # unflatten in the documented order
    p, off = [], 0
    shapes = [((F, cin, 3, 3), F)] + [((F, F, 3, 3), F)] * R + [((1, F, 3, 3), 1)]
    for ws, bs in shapes:
        nw = int(np.prod(ws))
        p.append((tt[off:off + nw].view(ws), tt[off + nw:off + nw + bs]))
        off += nw + bs
    a = torch.tensor(x)
    hcur = torch.relu(Fn.conv2d(a, p[0][0], p[0][1], padding=1))
    for k in range(1, R + 1):
        hcur = hcur + torch.relu(Fn.conv2d(hcur, p[k][0], p[k][1], padding=1))
    y = Fn.conv2d(hcur, p[-1][0], p[-1][1], padding=1)[:, 0]
    L = ((y - torch.tensor(t)) ** 2).mean()
    L.backward()
    assert np.max(np.abs(y.detach().numpy() - y_o)) <= 1e-12 * max(1, np.abs(y_o).max())
    assert abs(L.item() - L_o) <= 1e-13 * L_o
    gt = tt.grad.numpy()
    assert np.max(np.abs(gt - g_o)) <= 1e-12 * np.abs(gt).max()


def test_zero_residual_branches_reduce_to_two_convolutions():
    """With every residual layer zeroed, y = conv(relu(conv(x, W0) + b0), Wo) + bo,
    evaluated here with scipy's 2-D correlation."""
    from scipy.signal import correlate2d
    cin, F, R, n = 2, 3, 2, 6
    rng = np.random.default_rng(7)
    th = rand_net(rng, cin, F, R)
    o = F * cin * 9 + F
    th[o:o + R * (F * F * 9 + F)] = 0.0
    W0 = th[:F * cin * 9].reshape(F, cin, 3, 3)
    b0 = th[F * cin * 9:o]
    Wo = th[o + R * (F * F * 9 + F):-1].reshape(1, F, 3, 3)
    bo = th[-1]
    x = rng.standard_normal((1, cin, n, n))
    h0 = np.stack([sum(correlate2d(x[0, c], W0[f, c], mode="same") for c in range(cin)) + b0[f]
                   for f in range(F)])
    h0 = np.maximum(h0, 0)
    y = sum(correlate2d(h0[f], Wo[0, f], mode="same") for f in range(F)) + bo
    assert np.max(np.abs(O.cnn_forward(th, x, cin, F, R)[0] - y)) <= 1e-13


def test_centre_tap_network_is_the_identity_on_positive_input():
    cin, F, R, n = 1, 2, 2, 5
    th = np.zeros(O.cnn_nparams(cin, F, R))
    th[4] = 1.0                                   # W0[0][0][1][1]
    o_out = F * cin * 9 + F + R * (F * F * 9 + F)
    th[o_out + 4] = 1.0                           # Wo[0][0][1][1]
    x = np.abs(np.random.default_rng(1).standard_normal((1, 1, n, n)))
    assert np.array_equal(O.cnn_forward(th, x, cin, F, R)[0], x[0, 0])


def test_adam_first_step_closed_form():
    """From zero moments, bias correction makes the first step -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50) * np.logspace(-6, 3, 50)
    m, v = np.zeros(50), np.zeros(50)
    th1 = th.copy()
    O.adam(th1, g, m, v, 1, 1e-3)
    np.testing.assert_allclose(th1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    th2 = th1.copy()
    O.adam(th2, g, m, v, 2, 1e-3)
    np.testing.assert_allclose(th2, th1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_residual_loss_gradient_matches_central_differences():
    cin, F, R, n, B = 2, 3, 1, 6, 2
    rng = np.random.default_rng(13)
    th = rand_net(rng, cin, F, R)
    x = rng.standard_normal((B, cin, n, n))
    L, g = O.cnn_residual_loss_grad(th, x, cin, F, R)
    h = 1e-6
    for k in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (O.cnn_residual_loss_grad(tp, x, cin, F, R)[0] - O.cnn_residual_loss_grad(tm, x, cin, F, R)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_residual_loss_against_torch_with_an_independent_operator():
    """The residual loss rebuilt in torch: the FV operator from padded harmonic
    means (Dirichlet faces 2K, no-flow north/south), the network from conv2d."""
    torch = pytest.importorskip("torch")
    import torch.nn.functional as Fn
    cin, F, R, n, B = O.CNN_CIN, O.CNN_WIDTH, O.CNN_RES, 6, 2
    rng = np.random.default_rng(17)
    th = rand_net(rng, cin, F, R, 0.1)
    x = rng.standard_normal((B, cin, n, n))
    L_o, g_o = O.cnn_residual_loss_grad(th, x, cin, F, R)
    tt = torch.tensor(th, requires_grad=True)
    p, off = [], 0
    for ws, bs in [((F, cin, 3, 3), F)] + [((F, F, 3, 3), F)] * R + [((1, F, 3, 3), 1)]:
        nw = int(np.prod(ws))
        p.append((tt[off:off + nw].view(ws), tt[off + nw:off + nw + bs]))
        off += nw + bs
    a = torch.tensor(x)
    hcur = torch.relu(Fn.conv2d(a, p[0][0], p[0][1], padding=1))
    for k in range(1, R + 1):
        hcur = hcur + torch.relu(Fn.conv2d(hcur, p[k][0], p[k][1], padding=1))
    y = Fn.conv2d(hcur, p[-1][0], p[-1][1], padding=1)[:, 0]
    K = torch.exp(a[:, 0])
    hm = lambda u, v: 2 * u * v / (u + v)
    Tx = torch.cat([2 * K[:, :, :1], hm(K[:, :, :-1], K[:, :, 1:]), 2 * K[:, :, -1:]], dim=2)  # [B][n][n+1]
    z = torch.zeros_like(K[:, :1, :])
    Ty = torch.cat([z, hm(K[:, :-1, :], K[:, 1:, :]), z], dim=1)                          # [B][n+1][n]
    yp = Fn.pad(y, (1, 1, 1, 1))
    Ay = ((Tx[:, :, :-1] + Tx[:, :, 1:] + Ty[:, :-1, :] + Ty[:, 1:, :]) * y
          - Tx[:, :, :-1] * yp[:, 1:-1, :-2] - Tx[:, :, 1:] * yp[:, 1:-1, 2:]
          - Ty[:, :-1, :] * yp[:, :-2, 1:-1] - Ty[:, 1:, :] * yp[:, 2:, 1:-1])
    L = ((a[:, 1] - Ay) ** 2).mean()
    L.backward()
    assert abs(L.item() - L_o) <= 1e-13 * L_o
    gt = tt.grad.numpy()
    assert np.max(np.abs(gt - g_o)) <= 1e-12 * np.abs(gt).max()


def test_residual_loss_of_the_zero_network_is_the_mean_square_residual():
    rng = np.random.default_rng(19)
    x = rng.standard_normal((2, 2, 5, 5))
    L, _ = O.cnn_residual_loss_grad(np.zeros(O.cnn_nparams()), x)
    assert abs(L - np.mean(x[:, 1] ** 2)) <= 1e-15
