"""Straight-through gradient of log psi, FP64 (paper eqs. 7-8; Sec. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

The quantizer's forward value is the nearest codeword; the paper trains
through it with a straight-through estimator (eq. 7) whose backward follows
a softmax over the negative unsquared distances to all codewords (eq. 8).
This module writes that estimator as a relaxed surrogate, per quantizer
head h of every layer,

    V_h(theta) = W_h(theta)[c0] + (p(theta) - p(theta0))^T W_h(theta),
    p_j(theta) = softmax_j( -|| a_h(theta) - W_hj(theta) || ),

with the codes c0 fixed at their values at theta0.  Eq. (8) multiplies the
un-stopped codebook by g = SG[onehot] + softmax - SG[softmax]; the stop
gradient acts on the softmax output only, so the codebook's own factor in
V is the value of g, the one-hot vector.  At theta0 the surrogate's value is
the forward pass of ``oracle.network``; its true derivative there is the
straight-through gradient: the selected codeword receives the upstream
gradient through the one-hot factor, and every codeword and the attention
output a_h receive it through the distances inside the softmax (no
commitment loss).

The rest of the network is differentiated exactly.  Everything runs in
torch float64 on the CPU; gradients come from torch autograd.

Layout of the flat parameter vector and the network itself are those of
``oracle.network`` (Sec. 3.1); the codes are taken from its nearest-codeword
routine so that both agree bit for bit.
"""
import numpy as np
import torch

from . import network as onet

LN_EPS = onet.LN_EPS


def _unpack(cfg, th):
    """Views of the flat torch parameter vector th, in the flat layout."""
    d, Q, H, F = cfg.d_model, cfg.codebook_size, cfg.vq_heads, cfg.d_ff
    V, T = onet.classes(cfg), onet.n_tokens(cfg)
    enc = onet.encoder(cfg)
    pos = [0]

    def take(*shape):
        n = int(np.prod(shape))
        a = th[pos[0]:pos[0] + n].reshape(shape)
        pos[0] += n
        return a

    P = {"tok": take(V if enc else V + 1, d), "pos": take(T, d),
         "layers": []}
    for _ in range(cfg.n_layers):
        P["layers"].append(dict(
            ln1_g=take(d), ln1_b=take(d), W_qkv=take(d, 3 * d),
            b_qkv=take(3 * d), codebook=take(H, Q, d // H),
            W_o=take(d, d), b_o=take(d), ln2_g=take(d), ln2_b=take(d),
            W1=take(d, F), b1=take(F), W2=take(F, d), b2=take(d)))
    if getattr(cfg, "attn_tail", False):
        P["tail"] = dict(ln_g=take(d), ln_b=take(d), W_qkv=take(d, 3 * d),
                         b_qkv=take(3 * d), W_o=take(d, d), b_o=take(d))
    P["lnf_g"] = take(d)
    P["lnf_b"] = take(d)
    P["W_head"] = take(d, 1 if enc else V)
    P["b_head"] = take(1 if enc else V)
    assert pos[0] == th.numel()
    return P


def _ln(x, g, b):
    mu = x.mean(dim=-1, keepdim=True)
    var = ((x - mu) ** 2).mean(dim=-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + LN_EPS) * g + b


def _gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / np.sqrt(2.0)))


def _attention(q, k, v, n_heads, causal=True):
    S, N, d = q.shape
    dh = d // n_heads

    def heads(t):
        return t.reshape(S, N, n_heads, dh).transpose(1, 2)

    s = heads(q) @ heads(k).transpose(-1, -2) / np.sqrt(dh)
    if causal:
        mask = torch.triu(torch.ones(N, N, dtype=torch.bool), diagonal=1)
        s = s.masked_fill(mask, float("-inf"))
    p = torch.softmax(s, dim=-1)
    return (p @ heads(v)).transpose(1, 2).reshape(S, N, d)


def vq_surrogate(a, codebook, frozen=None):
    """Straight-through quantizer of a [S, N, d] (eqs. 7-8).

    Per head h: z_h = W_h[c] + (p - SG[p])^T W_h with p = softmax(-D_h),
    D_hj = ||a_h - W_hj|| (eq. 8, SG on the softmax only, the codebook
    factor live).  frozen: None for the autograd form (SG[p] is the detached
    softmax), else a dict with the codes and the softmax values at theta0
    (the finite-difference form, where p(theta0) is a constant).  Returns
    (z, codes, probs) with probs the detached softmax of every head."""
    H, Q, m = codebook.shape
    S, N, d = a.shape
    flat = a.reshape(S * N, d)
    if frozen is None:
        codes = np.stack([onet._nearest(flat[:, h * m:(h + 1) * m].detach()
                                        .numpy(), codebook[h].detach().numpy())[0]
                          for h in range(H)], axis=1)
    else:
        codes = frozen["codes"]
    segs, probs = [], []
    for h in range(H):
        seg = flat[:, h * m:(h + 1) * m]
        dist = torch.cdist(seg, codebook[h],
                           compute_mode="donot_use_mm_for_euclid_dist")
        p = torch.softmax(-dist, dim=-1)                 # eq. (8)
        p_sg = p.detach() if frozen is None else frozen["probs"][h]
        hard = codebook[h][torch.as_tensor(codes[:, h])]
        segs.append(hard + (p - p_sg) @ codebook[h])     # g(D)^T W, eq. (8)
        probs.append(p.detach())
    z = torch.cat(segs, dim=1).reshape(S, N, d)
    return z, codes, probs


def _forward(cfg, th, spins, frozen=None):
    """log psi [S] through the straight-through surrogate; also returns the
    per-layer frozen state (codes, softmax values) of this evaluation."""
    P = _unpack(cfg, th)
    t, u = onet.tokens(spins, onet.group(cfg))
    enc = onet.encoder(cfg)
    if enc:
        u = t                          # the encoder reads the tokens
    t = torch.as_tensor(t)
    u = torch.as_tensor(u)
    d = cfg.d_model
    x = P["tok"][u] + P["pos"][None]
    state = []
    for l, lay in enumerate(P["layers"]):
        h = _ln(x, lay["ln1_g"], lay["ln1_b"])
        qkv = h @ lay["W_qkv"] + lay["b_qkv"]
        a = _attention(qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:],
                       cfg.n_heads, causal=not enc)
        z, codes, probs = vq_surrogate(a, lay["codebook"],
                                       None if frozen is None else frozen[l])
        state.append({"codes": codes, "probs": probs})
        xp = x + z @ lay["W_o"] + lay["b_o"]
        hid = _gelu(_ln(xp, lay["ln2_g"], lay["ln2_b"]) @ lay["W1"] + lay["b1"])
        x = xp + hid @ lay["W2"] + lay["b2"]
    if "tail" in P:
        T = P["tail"]
        qkv = _ln(x, T["ln_g"], T["ln_b"]) @ T["W_qkv"] + T["b_qkv"]
        a = _attention(qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:],
                       cfg.n_heads)
        x = x + a @ T["W_o"] + T["b_o"]
    f = _ln(x, P["lnf_g"], P["lnf_b"])
    if enc:
        return (f @ P["W_head"])[..., 0].mean(dim=-1) + P["b_head"][0], state
    lp = torch.log_softmax(f @ P["W_head"] + P["b_head"], dim=-1)
    ell = torch.gather(lp, -1, t[..., None])[..., 0]
    return 0.5 * ell.sum(dim=-1), state


def logpsi(cfg, theta, spins):
    """log psi [S] of the surrogate at theta (equals the forward pass)."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64))
    with torch.no_grad():
        lp, _ = _forward(cfg, th, np.atleast_2d(spins))
    return lp.numpy()


def grad_logpsi(cfg, theta, spins, weights=None):
    """Straight-through gradient of log psi.

    weights None: per-sample gradients [S][P]; else the weighted sum
    sum_i w_i d log psi_i / d theta, shape [P]."""
    spins = np.atleast_2d(spins)
    theta = np.asarray(theta, dtype=np.float64)
    if weights is not None:
        th = torch.tensor(theta, requires_grad=True)
        lp, _ = _forward(cfg, th, spins)
        (lp * torch.as_tensor(np.asarray(weights, dtype=np.float64))).sum() \
            .backward()
        return th.grad.numpy().copy()
    out = np.empty((spins.shape[0], theta.size))
    for i in range(spins.shape[0]):
        th = torch.tensor(theta, requires_grad=True)
        lp, _ = _forward(cfg, th, spins[i:i + 1])
        lp.sum().backward()
        out[i] = th.grad.numpy()
    return out


def frozen_state(cfg, theta, spins):
    """Codes and softmax values at theta (for the finite-difference form)."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64))
    with torch.no_grad():
        _, st = _forward(cfg, th, np.atleast_2d(spins))
    return st


def surrogate_logpsi(cfg, theta, spins, frozen):
    """log psi [S] of the surrogate with the codes and the subtracted
    softmax held at their theta0 values (``frozen_state``): a smooth function
    of theta whose derivative at theta0 is the straight-through gradient."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64))
    with torch.no_grad():
        lp, _ = _forward(cfg, th, np.atleast_2d(spins), frozen=frozen)
    return lp.numpy()
