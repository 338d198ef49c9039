"""VQ transformer wave function, FP64 (paper Sec. 3.1 and Sec. 2).

Model (the readings of points the paper leaves open are listed in the
project's design notes; each is restated where it is used):

* The distribution network is an autoregressive decoder (Sec. 3.1) over
  tokens that are groups of K = cfg.group consecutive spins (K = 1: one
  token per spin).  Token t_i of group i is sum_k b_k 2^k with b_k = 1 for
  spin -1 at the group's k-th site (K = 1: 0 for +1, 1 for -1), one of
  2^K values.  The input at position i is the previous token (a
  beginning-of-sequence token 2^K at position 0), the target at position i
  is t_i, so P(s) = prod_i P(t_i | t_<i) (chain rule, Sec. 2) over the
  T = N / K tokens.
* Embedding: learned token + learned absolute position vectors.
* Each block (pre-LayerNorm):
      h  = LN1(x);  [q|k|v] = h W_qkv + b_qkv
      a  = causal multi-head self-attention (scale 1/sqrt(d_head))
      z  = VQ(a)   -- nearest codeword per quantizer head (eqs. 4-6)
      x' = x + z W_o + b_o      (VQ sits before the output projection and
                                 the residual, Sec. 3.1)
      x  = x' + W2 GELU(LN2(x') W1 + b1) + b2
* Optionally an attention-only half-block after the blocks (the paper's
  Table 1 networks end with one, with no quantizer): h = LN(x),
  [q|k|v] = h W_qkv + b, x = x + MHSA(q, k, v) W_o + b_o.
* Head: final LN, linear d -> 2^K, log-softmax; log P(s) = sum_i l_i.
* Zero phase (Sec. 4, Marshall-rotated Heisenberg), so
  log psi(s) = 1/2 log P(s)  (polar form of Sec. 2).
* The other network of Sec. 3.1, the bidirectional encoder (cfg.encoder),
  used as log psi: the same blocks over the tokens themselves (no shift,
  no beginning-of-sequence token) with attention over all positions; the
  last layer's hidden states are pooled (their mean after the final LN)
  and a linear map gives the scalar: log psi(s) = mean_i LN(x_i) . w + b.
  It is not autoregressive (no direct sampling).

Vector quantizer (eqs. 4-6): the input vector is split into H contiguous
segments; segment h picks the codeword of codebook W_h nearest in Euclidean
distance (the index that maximises D_hj = -||x_h - W_hj||); ties go to the
lowest index.  The value returned is the chosen codeword.
"""
import numpy as np
from scipy.special import erf

LN_EPS = 1e-5


def unpack(cfg, theta):
    """Split the flat FP64 parameter vector into named arrays (views)."""
    d, Q, H, F = cfg.d_model, cfg.codebook_size, cfg.vq_heads, cfg.d_ff
    V, T = classes(cfg), n_tokens(cfg)
    enc = encoder(cfg)
    if enc and getattr(cfg, "attn_tail", False):
        raise ValueError("the encoder has no attention-only half-block")
    theta = np.asarray(theta, dtype=np.float64)
    pos = [0]

    def take(*shape):
        n = int(np.prod(shape))
        a = theta[pos[0]:pos[0] + n].reshape(shape)
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
    if pos[0] != theta.size:
        raise ValueError(f"parameter vector has {theta.size} entries, "
                         f"model needs {pos[0]}")
    return P


def group(cfg):
    """Spins per token."""
    return getattr(cfg, "group", 1)


def classes(cfg):
    """Values of a token: 2^K."""
    return 1 << group(cfg)


def n_tokens(cfg):
    """Sequence length T = N / K."""
    if cfg.N % group(cfg):
        raise ValueError("the sites do not split into whole tokens")
    return cfg.N // group(cfg)


def encoder(cfg):
    """The bidirectional encoder with pooling in place of the decoder."""
    return bool(getattr(cfg, "encoder", False))


def n_params(cfg):
    d, Q, F = cfg.d_model, cfg.codebook_size, cfg.d_ff
    V, T = classes(cfg), n_tokens(cfg)
    if encoder(cfg):
        per_layer = (2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d
                     + d * F + F + F * d + d)
        return V * d + T * d + cfg.n_layers * per_layer + 2 * d + d + 1
    per_layer = (2 * d + d * 3 * d + 3 * d + Q * d + d * d + d + 2 * d
                 + d * F + F + F * d + d)
    tail = (2 * d + 3 * d * d + 3 * d + d * d + d
            if getattr(cfg, "attn_tail", False) else 0)
    return ((V + 1) * d + T * d + cfg.n_layers * per_layer + tail + 2 * d
            + d * V + V)


def tokens(spins, K=1):
    """Targets t [S, T] and shifted inputs u [S, T] (BOS = 2^K first) of
    spins [S, N] in tokens of K consecutive sites: t = sum_k b_k 2^k with
    b_k = 1 for spin -1 at the token's k-th site."""
    s = np.atleast_2d(np.asarray(spins))
    S, N = s.shape
    b = (s < 0).astype(np.int64).reshape(S, N // K, K)
    t = (b * (1 << np.arange(K, dtype=np.int64))).sum(axis=-1)
    u = np.concatenate([np.full((S, 1), 1 << K, dtype=np.int64),
                        t[:, :-1]], axis=1)
    return t, u


def layer_norm(x, g, b):
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)   # biased variance
    return (x - mu) / np.sqrt(var + LN_EPS) * g + b


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def causal_attention(q, k, v, n_heads, rows=None, causal=True):
    """Causal multi-head attention.

    q: [..., R, d] queries at sequence positions ``rows`` (default all N);
    k, v: [..., N, d].  Query at position i attends to keys j <= i
    (every key when causal is False: the bidirectional encoder).
    """
    N, d = k.shape[-2], k.shape[-1]
    R = q.shape[-2]
    dh = d // n_heads
    rows = np.arange(N) if rows is None else np.asarray(rows)
    masked = np.arange(N)[None, :] > rows[:, None]            # [R, N]
    if not causal:
        masked = np.zeros_like(masked)

    def heads(t, n):        # [..., n, d] -> [..., heads, n, dh]
        return np.swapaxes(t.reshape(t.shape[:-1] + (n_heads, dh)), -2, -3)

    qh, kh, vh = heads(q, R), heads(k, N), heads(v, N)
    s = qh @ np.swapaxes(kh, -1, -2) / np.sqrt(dh)             # [..., h, R, N]
    s = np.where(masked, -np.inf, s)
    s = s - s.max(axis=-1, keepdims=True)
    p = np.exp(s)
    p = p / p.sum(axis=-1, keepdims=True)
    o = p @ vh                                                 # [..., h, R, dh]
    return np.swapaxes(o, -2, -3).reshape(q.shape)


def _nearest(seg, cb):
    """Nearest codeword of cb [Q, m] for each row of seg [R, m].

    Candidates are screened with the expanded form |a|^2 - 2 a.w + |w|^2
    (one matrix product); the decision among all codes within a safe slack of
    the two smallest is then taken on squared differences summed directly.
    Returns (code, best distance, second-best distance), distances unsquared.
    """
    R, Q = seg.shape[0], cb.shape[0]
    a2 = (seg * seg).sum(axis=1)
    w2 = (cb * cb).sum(axis=1)
    approx = a2[:, None] - 2.0 * (seg @ cb.T) + w2[None, :]
    scale = a2 + w2.max() + 1.0
    code = np.empty(R, dtype=np.int64)
    d1 = np.empty(R)
    d2 = np.full(R, np.inf)
    if Q == 1:
        diff = seg - cb[0][None, :]
        code[:] = 0
        d1[:] = np.sqrt((diff * diff).sum(axis=1))
        return code, d1, d2
    top2 = np.argpartition(approx, 1, axis=1)[:, :2]          # two smallest
    second = np.take_along_axis(approx, top2, axis=1).max(axis=1)
    bound = second + 1e-9 * scale
    ncand = (approx <= bound[:, None]).sum(axis=1)
    # Rows with exactly two candidates: decide on direct squared differences.
    e0 = seg - cb[top2[:, 0]]
    e1 = seg - cb[top2[:, 1]]
    ex0 = (e0 * e0).sum(axis=1)
    ex1 = (e1 * e1).sum(axis=1)
    first_is_0 = (ex0 < ex1) | ((ex0 == ex1) & (top2[:, 0] < top2[:, 1]))
    code[:] = np.where(first_is_0, top2[:, 0], top2[:, 1])
    d1[:] = np.sqrt(np.where(first_is_0, ex0, ex1))
    d2[:] = np.sqrt(np.where(first_is_0, ex1, ex0))
    # Rows with more near-equal candidates: full direct comparison.
    for r in np.nonzero(ncand > 2)[0]:
        cand = np.nonzero(approx[r] <= bound[r])[0]          # ascending ids
        diff = seg[r][None, :] - cb[cand]
        ex = (diff * diff).sum(axis=1)
        order = np.argsort(ex, kind="stable")                # lowest id on ties
        code[r] = cand[order[0]]
        d1[r] = np.sqrt(ex[order[0]])
        d2[r] = np.sqrt(ex[order[1]])
    return code, d1, d2


def quantize(a, codebook):
    """Multi-head VQ of a [..., d] with codebook [H, Q, d/H].

    Returns codes [..., H], quantized vectors z [..., d], and the best and
    second-best unsquared distances d1, d2 [..., H].
    """
    H, Q, m = codebook.shape
    lead = a.shape[:-1]
    flat = a.reshape(-1, a.shape[-1])
    codes = np.empty((flat.shape[0], H), dtype=np.int64)
    d1 = np.empty((flat.shape[0], H))
    d2 = np.empty((flat.shape[0], H))
    z = np.empty_like(flat)
    for h in range(H):
        seg = flat[:, h * m:(h + 1) * m]
        c, b1, b2 = _nearest(seg, codebook[h])
        codes[:, h] = c
        d1[:, h] = b1
        d2[:, h] = b2
        z[:, h * m:(h + 1) * m] = codebook[h][c]
    return (codes.reshape(lead + (H,)), z.reshape(a.shape),
            d1.reshape(lead + (H,)), d2.reshape(lead + (H,)))


def qkv_rows(lay, x):
    h = layer_norm(x, lay["ln1_g"], lay["ln1_b"])
    return h @ lay["W_qkv"] + lay["b_qkv"]


def post_vq_rows(lay, x, z):
    """Output projection + residual, then the MLP sub-block (per location)."""
    xp = x + z @ lay["W_o"] + lay["b_o"]
    hid = gelu(layer_norm(xp, lay["ln2_g"], lay["ln2_b"]) @ lay["W1"]
               + lay["b1"])
    return xp + hid @ lay["W2"] + lay["b2"]


def tail_block(T, x, n_heads):
    """The attention-only half-block: pre-LN causal self-attention and
    the output projection with its residual, no quantizer, no MLP."""
    d = x.shape[-1]
    qkv = layer_norm(x, T["ln_g"], T["ln_b"]) @ T["W_qkv"] + T["b_qkv"]
    a = causal_attention(qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:],
                         n_heads)
    return x + a @ T["W_o"] + T["b_o"]


def head_logprobs(P, x):
    """Log-probabilities of every token value at every position,
    [..., 2^K]."""
    f = layer_norm(x, P["lnf_g"], P["lnf_b"])
    logits = f @ P["W_head"] + P["b_head"]
    m = logits.max(axis=-1, keepdims=True)
    return logits - (m + np.log(np.exp(logits - m).sum(axis=-1,
                                                         keepdims=True)))


def pooled_terms(P, x):
    """Encoder head: every position's LN(x_i) . w, [..., T]; log psi is
    their mean plus the bias."""
    f = layer_norm(x, P["lnf_g"], P["lnf_b"])
    return (f @ P["W_head"])[..., 0]


def forward(cfg, P, spins, keep=False):
    """Full forward pass of a batch of sequences spins [S, N].

    Returns a dict with ``logpsi`` [S], per-position target log-probs
    ``ell`` [S, T], the log-probs of every token value ``lp`` [S, T, 2^K],
    per-layer codes ``codes`` [n_layers, S, T, H]; with keep=True also
    per-layer caches (block input x, q, k, v, attention output a, d1, d2).
    T = N / K positions (K = 1: one per site).
    """
    spins = np.atleast_2d(spins)
    t, u = tokens(spins, group(cfg))
    enc = encoder(cfg)
    if enc:
        u = t                          # the encoder reads the tokens
    d = cfg.d_model
    x = P["tok"][u] + P["pos"][None, :, :]
    codes, caches = [], []
    for lay in P["layers"]:
        qkv = qkv_rows(lay, x)
        q, k, v = qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:]
        a = causal_attention(q, k, v, cfg.n_heads, causal=not enc)
        c, z, d1, d2 = quantize(a, lay["codebook"])
        if keep:
            caches.append(dict(x=x, q=q, k=k, v=v, a=a, codes=c, d1=d1,
                               d2=d2))
        x = post_vq_rows(lay, x, z)
        codes.append(c)
    tail_cache = None
    if "tail" in P:
        if keep:
            T = P["tail"]
            qkv = qkv_rows(dict(ln1_g=T["ln_g"], ln1_b=T["ln_b"],
                                W_qkv=T["W_qkv"], b_qkv=T["b_qkv"]), x)
            tail_cache = dict(x=x, q=qkv[..., :d], k=qkv[..., d:2 * d],
                              v=qkv[..., 2 * d:])
        x = tail_block(P["tail"], x, cfg.n_heads)
    if enc:
        c = pooled_terms(P, x)
        out = dict(logpsi=c.mean(axis=-1) + P["b_head"][0], terms=c,
                   ell=None, lp=None,
                   codes=np.stack(codes) if codes else None, x_final=x)
        if keep:
            out["caches"] = caches
            out["tail"] = None
        return out
    lp = head_logprobs(P, x)
    ell = np.take_along_axis(lp, t[..., None], axis=-1)[..., 0]
    out = dict(logpsi=0.5 * ell.sum(axis=-1), ell=ell, lp=lp,
               codes=np.stack(codes) if codes else None, x_final=x)
    if keep:
        out["caches"] = caches
        out["tail"] = tail_cache
    return out


def logpsi_fn(cfg, P, chunk=64):
    """Batched log psi callable for the local-energy routines."""
    def f(spins):
        spins = np.atleast_2d(spins)
        out = np.empty(spins.shape[0])
        for s in range(0, spins.shape[0], chunk):
            out[s:s + chunk] = forward(cfg, P, spins[s:s + chunk])["logpsi"]
        return out
    return f
