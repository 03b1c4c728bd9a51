"""The allocation-free perceptron gradient (nb_mlp_grad_static) against the
allocating one (nb_mlp_grad) and the FP64 oracle, through the C ABI.

Two calls in a row share the per-GPU static scratch; the second has fewer
rows, so any value the first call left behind that the second read would
show up as a mismatch."""
import sys

import numpy as np
import pytest

import oracle
import paper_1907_02290_amd as nb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(nb.MLP_NPARAM) * scale).astype(np.float32)


def _data(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 12)).astype(np.float32)
    y = (rng.uniform(size=n) > 0.7).astype(np.float32)
    return x, y


def _static_grad(ctx, x, y, pw):
    dev = torch.device("cuda", 0)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    g = torch.full((nb.MLP_NPARAM,), float("nan"), dtype=torch.float32,
                   device=dev)
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    ctx.mlp_grad_static(xd, yd, g, loss, pos_weight=pw)
    torch.cuda.synchronize()
    return float(loss.cpu()[0]), g.cpu().numpy()


def test_static_gradient_matches_allocating_gradient_and_oracle():
    assert torch.cuda.is_available()
    w = _weights(11)
    with nb.Context() as ctx:
        ctx.mlp_set(w)
        # two calls in a row on the shared scratch, the second smaller
        for n, pw, seed in ((nb.MLP_STATIC_MAX_ROWS, 3.0, 12), (777, 1.0, 13)):
            say("case static gradient n=%d pos_weight=%g" % (n, pw))
            x, y = _data(seed, n)
            sl, sg = _static_grad(ctx, x, y, pw)
            al, ag = ctx.mlp_grad(x, y, pos_weight=pw)
            # same kernels, same summation order: identical bits
            np.testing.assert_array_equal(sg, ag)
            assert sl == al
            ol, og = oracle.mlp_loss_grad(w.astype(np.float64), x, y, pw)
            assert abs(sl - ol) <= 1e-4 * max(1.0, abs(ol))
            assert np.max(np.abs(sg - og)) <= 1e-4 * np.max(np.abs(og))


def test_static_gradient_without_loss_pointer_and_a_second_context():
    w = _weights(21)
    x, y = _data(22, 1500)
    dev = torch.device("cuda", 0)
    with nb.Context() as a, nb.Context() as b:
        a.mlp_set(w)
        b.mlp_set(w)
        g1 = torch.zeros(nb.MLP_NPARAM, dtype=torch.float32, device=dev)
        g2 = torch.zeros_like(g1)
        xd = torch.from_numpy(x).to(dev)
        yd = torch.from_numpy(y).to(dev)
        torch.cuda.synchronize()
        a.mlp_grad_static(xd, yd, g1)
        torch.cuda.synchronize()
        b.mlp_grad_static(xd, yd, g2, pos_weight=1.0)
        torch.cuda.synchronize()
        _, ref = a.mlp_grad(x, y)
        np.testing.assert_array_equal(g1.cpu().numpy(), ref)
        np.testing.assert_array_equal(g2.cpu().numpy(), ref)


def test_static_gradient_rejects_what_it_cannot_hold():
    dev = torch.device("cuda", 0)
    lib = nb.load()
    with nb.Context() as ctx:
        x = torch.zeros((16, 12), dtype=torch.float32, device=dev)
        y = torch.zeros(16, dtype=torch.float32, device=dev)
        g = torch.zeros(nb.MLP_NPARAM, dtype=torch.float32, device=dev)
        # no weights yet
        with pytest.raises(nb.NbError) as e:
            ctx.mlp_grad_static(x, y, g)
        assert e.value.code == nb.NB_ERR_STATE
        ctx.mlp_set(_weights(31))
        h = ctx._h
        px, py, pg = x.data_ptr(), y.data_ptr(), g.data_ptr()
        too_many = nb.MLP_STATIC_MAX_ROWS + 1
        assert lib.nb_mlp_grad_static(h, too_many, px, py, 1.0, None,
                                      pg) == nb.NB_ERR_INPUT
        assert lib.nb_mlp_grad_static(h, 0, px, py, 1.0, None,
                                      pg) == nb.NB_ERR_INPUT
        assert lib.nb_mlp_grad_static(h, 16, px, py, 1.0, None,
                                      None) == nb.NB_ERR_INPUT
        assert lib.nb_mlp_grad_static(h, 16, px, py, 0.0, None,
                                      pg) == nb.NB_ERR_INPUT
        assert lib.nb_mlp_grad_static(h, 16, px, py, 1.0, None, pg) == nb.NB_OK
        torch.cuda.synchronize()
