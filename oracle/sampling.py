"""Direct (exact) sampling from the autoregressive wave function, FP64
(paper Sec. 2: psi(s)^2 = P(s) = prod_i P(s_i | s_<i) supports sampling
site by site at the cost of evaluating P).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Site i of every sample is drawn from the network's conditional
P(s_i = +1 | s_<i) given the sites already drawn: s_i = +1 exactly when the
caller's uniform number u_i is below that probability.  The conditional of
site i is read from a full forward pass of the partial sequence; the sites
after i do not influence it (causal attention, inputs shifted by one site),
so they are filled with +1 placeholders.  This is the definition written
out, one forward pass per site.
"""
import numpy as np

from . import network as net


def sample(cfg, theta, uniforms):
    """Samples spins [S, N] (int8) for uniforms [S, N] in [0, 1).

    Returns (spins, logpsi, p_up): log psi = 1/2 sum_i log P(s_i | s_<i)
    over the drawn conditionals, and p_up [S, N] the conditional
    probabilities of +1 the draws compared against."""
    P = net.unpack(cfg, theta)
    u = np.asarray(uniforms, dtype=np.float64)
    S, N = u.shape
    if N != cfg.N:
        raise ValueError("uniforms must have one column per site")
    s = np.ones((S, N), dtype=np.int8)
    ell = np.zeros((S, N))
    p_up = np.zeros((S, N))
    for i in range(N):
        lp = net.forward(cfg, P, s)["lp"][:, i, :]     # [S, 2] log-probs
        p = np.exp(lp[:, 0])                           # P(s_i = +1 | s_<i)
        up = u[:, i] < p
        s[:, i] = np.where(up, 1, -1)
        ell[:, i] = np.where(up, lp[:, 0], lp[:, 1])
        p_up[:, i] = p
    logpsi = np.zeros(S)
    for i in range(N):                                 # site order
        logpsi += ell[:, i]
    return s, 0.5 * logpsi, p_up
