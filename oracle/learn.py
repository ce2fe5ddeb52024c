"""FP64 oracle of the learning-episode update (TEST INFRASTRUCTURE ONLY): the steps of the
SHAC algorithm that follow a window (Sec. 3.3, Algorithm "SHAC" and Eqs. "critic_loss" and
"td-lambda"), written in their defining form.

* td_lambda: the estimate of Eq. "td-lambda", the lambda-weighted average of the k-step
  returns G_t^k = sum_{l<k} gamma^l r_{t+l} + gamma^k V(s_{t+k}), summed term by term.
* adam_step: Adam (Kingma and Ba) with bias-corrected moments.
* critic_fit: the mean squared error of Eq. "critic_loss" over each minibatch of a shuffled
  pass, its gradient by reverse mode, one Adam step per minibatch.
* soft_update: the target critic update of the algorithm, alpha V' + (1 - alpha) V.
"""
import torch

from .window import mlp_forward

F64 = torch.float64


def _t(x):
    return x.detach().to(F64) if torch.is_tensor(x) else torch.as_tensor(x, dtype=F64)


def td_lambda(rewards, values, gamma, lam, done=None):
    """rewards [h, N], values [h+1, N] (V(s_0) .. V(s_h)) -> estimates [h, N].

    done [h, N] (optional) marks frames that ended in early termination: a k-step return
    G_t^k that reaches such a frame t + j (j < k) stops there, with the rewards up to
    r_{t+j} and no value (the failed state is worth nothing), so G_t^k = G_t^{j+1} for
    every longer k."""
    r, v = _t(rewards), _t(values)
    h, N = r.shape
    dn = torch.zeros(h, N, dtype=torch.bool) if done is None else torch.as_tensor(done).bool()
    out = torch.zeros_like(r)
    for t in range(h):
        n = h - t
        # d[e]: offset of the first terminated frame from t (n if none inside the window)
        d = torch.full((N,), n, dtype=torch.long)
        for j in reversed(range(n)):
            d = torch.where(dn[t + j], torch.full_like(d, j), d)

        def G(k):
            full = sum(gamma ** l * r[t + l] for l in range(k)) + gamma ** k * v[t + k]
            cut = sum(gamma ** l * r[t + l] * (l <= d) for l in range(k))
            return torch.where(k > d, cut, full)
        est = sum((1.0 - lam) * lam ** (k - 1) * G(k) for k in range(1, n))
        out[t] = est + lam ** (n - 1) * G(n)
    return out


def obs_stats_update(obs, count, mean, var, eps):
    """Running observation statistics (Sec. 3.3): the mean and population variance of every
    observation seen so far, from the first and second raw moments of the union of the
    `count` earlier samples (summarised by mean and var) and the new rows obs [rows, dim].
    Returns (count', mean', var', inv_std = 1 / sqrt(var' + eps))."""
    x = _t(obs)
    rows = x.shape[0]
    n = count + rows
    m0 = _t(mean) if count > 0 else torch.zeros(x.shape[1], dtype=torch.float64)
    v0 = _t(var) if count > 0 else torch.zeros(x.shape[1], dtype=torch.float64)
    first = (count * m0 + x.sum(0)) / n
    second = (count * (v0 + m0 * m0) + (x * x).sum(0)) / n
    v = second - first * first
    return n, first, v, 1.0 / torch.sqrt(v + eps)


def adam_step(params, grads, m, v, step, lr, beta1, beta2, eps):
    """One Adam step; returns (params, m, v) as new lists."""
    P, M, V = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        p, g, mm, vv = _t(p), _t(g), _t(mm), _t(vv)
        mm = beta1 * mm + (1.0 - beta1) * g
        vv = beta2 * vv + (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** step)
        vhat = vv / (1.0 - beta2 ** step)
        P.append(p - lr * mhat / (torch.sqrt(vhat) + eps))
        M.append(mm)
        V.append(vv)
    return P, M, V


def soft_update(target, online, alpha):
    return [alpha * _t(a) + (1.0 - alpha) * _t(b) for a, b in zip(target, online)]


def critic_values(layers, obs, ln=None):
    """V(obs); ln: None, or per hidden layer the (gain, bias) of its layer normalisation."""
    lnt = None if ln is None else [(_t(g), _t(b)) for g, b in ln]
    return mlp_forward([(_t(W), _t(b)) for W, b in layers], _t(obs), ln=lnt)[:, 0]


def _flat_params(layers, ln):
    """The critic's parameters in the library's order: per layer W, b, and after a hidden
    layer's W, b its normalisation gain and bias (with ln)."""
    out = []
    for i, (W, b) in enumerate(layers):
        out += [_t(W), _t(b)]
        if ln is not None and i < len(layers) - 1:
            out += [_t(ln[i][0]), _t(ln[i][1])]
    return out


def _unflat(params, n_layers, with_ln):
    layers, ln, k = [], [], 0
    for i in range(n_layers):
        layers.append((params[k], params[k + 1]))
        k += 2
        if with_ln and i < n_layers - 1:
            ln.append((params[k], params[k + 1]))
            k += 2
    return layers, (ln if with_ln else None)


def critic_fit(layers, obs, targets, perm, n_minibatch, m, v, adam_step0, lr, beta1, beta2, eps, ln=None):
    """layers [(W, b)], obs [rows, od], targets [rows], perm [n_iter, rows]; m, v lists shaped
    like the parameters in the library's order (W_0, b_0, [g_0, beta_0,] W_1, ...); ln: None or
    the (gain, bias) of each hidden layer's normalisation, fitted with the weights.
    Returns (layers, m, v, losses), and with ln (layers, ln, m, v, losses)."""
    n_layers = len(layers)
    params = _flat_params(layers, ln)
    m = [_t(x) for x in m]
    v = [_t(x) for x in v]
    obs, targets = _t(obs), _t(targets)
    rows = obs.shape[0]
    step = adam_step0
    losses = []
    for it in range(len(perm)):
        for mb in range(n_minibatch):
            idx = torch.as_tensor(perm[it][mb * rows // n_minibatch:(mb + 1) * rows // n_minibatch], dtype=torch.long)
            ps = [p.clone().requires_grad_(True) for p in params]
            lay, lnp = _unflat(ps, n_layers, ln is not None)
            V = mlp_forward(lay, obs[idx], ln=lnp)[:, 0]
            loss = ((V - targets[idx]) ** 2).mean()
            grads = torch.autograd.grad(loss, ps)
            losses.append(float(loss.detach()))
            step += 1
            params, m, v = adam_step(params, grads, m, v, step, lr, beta1, beta2, eps)
    lay, lnp = _unflat(params, n_layers, ln is not None)
    if ln is None:
        return lay, m, v, losses
    return lay, lnp, m, v, losses
