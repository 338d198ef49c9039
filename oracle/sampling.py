"""Direct (exact) sampling from the autoregressive wave function, FP64
(paper Sec. 2: psi(s)^2 = P(s) = prod_i P(t_i | t_<i) supports sampling
token by token at the cost of evaluating P).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One spin per token (K = 1): site i of every sample is drawn from the
network's conditional P(s_i = +1 | s_<i) given the sites already drawn:
s_i = +1 exactly when the caller's uniform number u_i is below that
probability.  Tokens of K > 1 spins: token i takes the smallest value c
whose cumulative probability P(t_i <= c | t_<i) (values in increasing
order, summed in that order) exceeds the uniform number of the token's
first site, u[iK]; its K spins follow from the bits of c.  The conditional
is read from a full forward pass of the partial sequence; the positions
after i do not influence it (causal attention, inputs shifted by one
token), so they are filled with +1 placeholders.  This is the definition
written out, one forward pass per token.
"""
import numpy as np

from . import network as net


def sample(cfg, theta, uniforms):
    """Samples spins [S, N] (int8) for uniforms [S, N] in [0, 1).

    Returns (spins, logpsi, probs): log psi = 1/2 sum_i log P(t_i | t_<i)
    over the drawn conditionals; probs are what the draws compared against:
    [S, N] conditional probabilities of +1 for K = 1, [S, T, 2^K] the
    conditional probabilities of every token value for K > 1."""
    if net.encoder(cfg):
        raise ValueError("the bidirectional encoder is not autoregressive: "
                         "no direct sampling")
    P = net.unpack(cfg, theta)
    u = np.asarray(uniforms, dtype=np.float64)
    S, N = u.shape
    if N != cfg.N:
        raise ValueError("uniforms must have one column per site")
    K, V, T = net.group(cfg), net.classes(cfg), net.n_tokens(cfg)
    s = np.ones((S, N), dtype=np.int8)
    ell = np.zeros((S, T))
    probs = np.zeros((S, N)) if K == 1 else np.zeros((S, T, V))
    for i in range(T):
        lp = net.forward(cfg, P, s)["lp"][:, i, :]     # [S, 2^K] log-probs
        if K == 1:
            p = np.exp(lp[:, 0])                       # P(s_i = +1 | s_<i)
            up = u[:, i] < p
            s[:, i] = np.where(up, 1, -1)
            ell[:, i] = np.where(up, lp[:, 0], lp[:, 1])
            probs[:, i] = p
            continue
        p = np.exp(lp)
        cdf = np.zeros(S)
        c = np.full(S, V - 1)
        done = np.zeros(S, dtype=bool)
        for v in range(V):                             # increasing values
            cdf = cdf + p[:, v]
            hit = ~done & (u[:, i * K] < cdf)
            c[hit] = v
            done |= hit
        for k in range(K):
            s[:, i * K + k] = np.where((c >> k) & 1, -1, 1)
        ell[:, i] = lp[np.arange(S), c]
        probs[:, i] = p
    logpsi = np.zeros(S)
    for i in range(T):                                 # token order
        logpsi += ell[:, i]
    return s, 0.5 * logpsi, probs
