"""Pins of the learning-episode oracle (TD-lambda, Adam, critic fit) against textbook
special cases and finite differences."""
import numpy as np
import torch

from oracle.learn import td_lambda, adam_step, critic_fit, critic_values, obs_stats_update


def test_td_lambda_special_cases():
    rng = np.random.default_rng(5)
    h, N, g = 7, 3, 0.9
    r = rng.normal(size=(h, N))
    v = rng.normal(size=(h + 1, N))
    # lambda = 0: one-step temporal difference target
    np.testing.assert_allclose(td_lambda(r, v, g, 0.0).numpy(), r + g * v[1:], rtol=0, atol=1e-13)
    # lambda = 1: the discounted return to the end of the window, bootstrapped there
    mc = np.stack([sum(g ** l * r[t + l] for l in range(h - t)) + g ** (h - t) * v[h] for t in range(h)])
    np.testing.assert_allclose(td_lambda(r, v, g, 1.0).numpy(), mc, rtol=0, atol=1e-12)
    # one frame: r_0 + gamma V(s_1) for any lambda
    np.testing.assert_allclose(td_lambda(r[:1], v[:2], g, 0.37).numpy(), r[:1] + g * v[1:2], atol=1e-14)


def test_td_lambda_with_termination():
    """Termination flags (App. A.3 heights; Sec. 3.3 resets): every return from a frame that
    ended in termination stops there with no value."""
    rng = np.random.default_rng(8)
    h, N, g = 6, 4, 0.9
    r = rng.normal(size=(h, N))
    v = rng.normal(size=(h + 1, N))
    done = np.zeros((h, N), bool)
    done[2, 0] = True                         # env 0 fails in frame 2
    done[0, 1] = done[4, 1] = True            # env 1 twice
    done[:, 2] = True                         # env 2 in every frame
    # lambda = 0: r_t + gamma V(s_{t+1}), without the value after a failed frame
    np.testing.assert_allclose(td_lambda(r, v, g, 0.0, done).numpy(), r + g * v[1:] * ~done, rtol=0, atol=1e-13)
    # lambda = 1: the discounted return to the first failure (inclusive) or to the window's
    # end, bootstrapped only there
    mc = np.zeros((h, N))
    for e in range(N):
        for t in range(h):
            acc, k = 0.0, t
            while True:
                acc += g ** (k - t) * r[k, e]
                if done[k, e]:
                    break
                k += 1
                if k == h:
                    acc += g ** (h - t) * v[h, e]
                    break
            mc[t, e] = acc
    np.testing.assert_allclose(td_lambda(r, v, g, 1.0, done).numpy(), mc, rtol=0, atol=1e-12)
    out = td_lambda(r, v, g, 0.8, done).numpy()
    np.testing.assert_allclose(out[:, 2], r[:, 2], rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[:, 3], td_lambda(r[:, 3:], v[:, 3:], g, 0.8).numpy()[:, 0], rtol=0, atol=1e-15)
    # frames up to a failure do not see what comes after it
    r2, v2 = r.copy(), v.copy()
    r2[3:, 0] += 5.0
    v2[3:, 0] -= 7.0
    np.testing.assert_array_equal(td_lambda(r2, v2, g, 0.8, done).numpy()[:3, 0], out[:3, 0])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(6)
    p = [torch.as_tensor(rng.normal(size=(4, 3)))]
    gr = [torch.as_tensor(rng.normal(size=(4, 3)))]
    z = [torch.zeros(4, 3, dtype=torch.float64)]
    P, M, V = adam_step(p, gr, z, z, 1, 0.01, 0.7, 0.95, 1e-8)
    # bias-corrected first moments are g and g^2: the step is lr g / (|g| + eps)
    np.testing.assert_allclose(P[0].numpy(), (p[0] - 0.01 * gr[0] / (gr[0].abs() + 1e-8)).numpy(), atol=1e-15)
    np.testing.assert_allclose(M[0].numpy(), 0.3 * gr[0].numpy(), atol=1e-15)
    np.testing.assert_allclose(V[0].numpy(), 0.05 * gr[0].numpy() ** 2, atol=1e-15)


def test_critic_fit_gradient_direction_and_descent():
    rng = np.random.default_rng(7)
    od, rows = 5, 24
    layers = [(rng.normal(0, 0.4, (8, od)), rng.normal(0, 0.1, 8)),
              (rng.normal(0, 0.4, (1, 8)), rng.normal(0, 0.1, 1))]
    obs = rng.normal(size=(rows, od))
    tgt = rng.normal(size=rows)
    zeros = [np.zeros_like(x) for W, b in layers for x in (W, b)]
    perm = [np.arange(rows)]
    new, _, _, losses = critic_fit(layers, obs, tgt, perm, 1, zeros, zeros, 0, 1e-7, 0.7, 0.95, 1e-12)

    def loss(Ls):
        return float(((critic_values(Ls, obs) - torch.as_tensor(tgt)) ** 2).mean())
    assert abs(losses[0] - loss(layers)) < 1e-14
    # the first Adam step moves every weight against the sign of its gradient: compare
    # with central differences of the loss on a few weights
    e = 1e-6
    for (i, j, k) in [(0, 0, 0), (0, 3, 2), (1, 0, 5)]:
        Lp = [(W.copy(), b.copy()) for W, b in layers]
        Lm = [(W.copy(), b.copy()) for W, b in layers]
        Lp[i][0][j, k] += e
        Lm[i][0][j, k] -= e
        fd = (loss(Lp) - loss(Lm)) / (2 * e)
        step = float(new[i][0][j, k]) - layers[i][0][j, k]
        assert np.sign(step) == -np.sign(fd) and abs(fd) > 1e-9
    # and a few passes with a usable rate reduce the loss
    perm = [rng.permutation(rows) for _ in range(30)]
    _, _, _, losses = critic_fit(layers, obs, tgt, perm, 2, zeros, zeros, 0, 1e-2, 0.7, 0.95, 1e-8)
    assert np.mean(losses[-2:]) < 0.75 * np.mean(losses[:2])


def test_critic_fit_with_layer_norm_follows_the_loss_gradient():
    """The critic fit with layer normalisation (App. A.2) on every hidden layer: with zero
    moments and an Adam epsilon far above every gradient, the first step moves each
    parameter by -lr g / (|g| + eps), so (lr = eps) the step is -g to a relative 1e-6; every
    weight, bias, gain and normalisation bias (in the library's order W, b, g, beta per hidden
    layer) is held to central differences of the minibatch loss."""
    rng = np.random.default_rng(17)
    od, rows = 5, 16
    layers = [(rng.normal(0, 0.4, (6, od)), rng.normal(0, 0.1, 6)),
              (rng.normal(0, 0.4, (4, 6)), rng.normal(0, 0.1, 4)),
              (rng.normal(0, 0.4, (1, 4)), rng.normal(0, 0.1, 1))]
    ln = [(rng.uniform(0.5, 1.5, 6), rng.normal(0, 0.2, 6)), (rng.uniform(0.5, 1.5, 4), rng.normal(0, 0.2, 4))]
    obs = rng.normal(size=(rows, od))
    tgt = rng.normal(size=rows)
    flat = [W for W in (layers[0][0], layers[0][1], ln[0][0], ln[0][1], layers[1][0], layers[1][1], ln[1][0],
                        ln[1][1], layers[2][0], layers[2][1])]
    zeros = [np.zeros_like(x) for x in flat]
    big = 1e6
    new_layers, new_ln, _, _, losses = critic_fit(layers, obs, tgt, [np.arange(rows)], 1, zeros, zeros, 0, big,
                                                  0.7, 0.95, big, ln=ln)
    new_flat = [new_layers[0][0], new_layers[0][1], new_ln[0][0], new_ln[0][1], new_layers[1][0],
                new_layers[1][1], new_ln[1][0], new_ln[1][1], new_layers[2][0], new_layers[2][1]]

    def loss(fl):
        Ls = [(fl[0], fl[1]), (fl[4], fl[5]), (fl[8], fl[9])]
        lnp = [(fl[2], fl[3]), (fl[6], fl[7])]
        return float(((critic_values(Ls, obs, ln=lnp) - torch.as_tensor(tgt)) ** 2).mean())
    assert abs(losses[0] - loss(flat)) < 1e-14
    e = 1e-6
    for t, x in enumerate(flat):
        for idx in [(0,) * x.ndim, tuple(s - 1 for s in x.shape)]:
            fp = [y.copy() for y in flat]
            fm = [y.copy() for y in flat]
            fp[t][idx] += e
            fm[t][idx] -= e
            fd = (loss(fp) - loss(fm)) / (2 * e)
            g = -(float(new_flat[t][idx]) - x[idx])
            assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-3), (t, idx, g, fd)


def test_obs_stats_streaming_equals_batch_moments():
    """Running observation statistics (Sec. 3.3) merged over uneven chunks equal the mean and
    population variance of all rows at once (numpy), and inv_std follows from them."""
    rng = np.random.default_rng(9)
    dim = 7
    chunks = [rng.normal(loc=rng.normal(size=dim), scale=rng.uniform(0.2, 3.0, dim), size=(n, dim))
              for n in (5, 1, 40, 13)]
    count, mean, var = 0, None, None
    for c in chunks:
        count, mean, var, inv = obs_stats_update(c, count, mean, var, 1e-5)
    allx = np.concatenate(chunks)
    assert count == allx.shape[0]
    np.testing.assert_allclose(mean.numpy(), allx.mean(0), rtol=0, atol=1e-13)
    np.testing.assert_allclose(var.numpy(), allx.var(0), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(inv.numpy(), 1.0 / np.sqrt(allx.var(0) + 1e-5), rtol=1e-12)
    # a constant column has zero variance and inv_std 1 / sqrt(eps)
    cnt, m1, v1, i1 = obs_stats_update(np.full((6, 2), 3.5), 0, None, None, 1e-4)
    np.testing.assert_allclose(m1.numpy(), [3.5, 3.5], rtol=0, atol=1e-15)
    np.testing.assert_allclose(v1.numpy(), [0.0, 0.0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(i1.numpy(), [100.0, 100.0], rtol=1e-9)
