"""Flat parameter layout of the VQ transformer (storage order, row-major).

Every weight matrix is stored [in][out] and applied as x @ W.  A token is a
group of K consecutive spins (K = cfg.group); its id is sum_k b_k 2^k with
b_k = 1 for spin -1 of the group's k-th site, and id 2^K is the
beginning-of-sequence token (K = 1: 0 = spin +1, 1 = spin -1, 2 = BOS).
T = N / K tokens.

  tok_emb[2^K + 1][d]  pos_emb[T][d]
  per layer:
    ln1_g[d] ln1_b[d]  W_qkv[d][3d] b_qkv[3d]  codebook[H][Q][d/H]
    W_o[d][d] b_o[d]   ln2_g[d] ln2_b[d]
    W1[d][d_ff] b1[d_ff]  W2[d_ff][d] b2[d]
  attention-only half-block (when the model has one):
    tail.ln_g[d] tail.ln_b[d]  tail.W_qkv[d][3d] tail.b_qkv[3d]
    tail.W_o[d][d] tail.b_o[d]
  lnf_g[d] lnf_b[d]  W_head[d][2^K] b_head[2^K]

The bidirectional encoder (cfg.encoder) reads the tokens themselves, with no
beginning-of-sequence token: tok_emb[2^K][d]; its head is one output,
W_head[d][1] b_head[1], averaged over the positions (log psi).

Each entry carries a ``kind`` tag used only by the seeded initialiser:
"w" (Gaussian), "gain" (set to 1) or "bias" (set to 0).
"""


def param_layout(cfg):
    d, Q, H, F = cfg.d_model, cfg.codebook_size, cfg.vq_heads, cfg.d_ff
    V = 1 << getattr(cfg, "group", 1)        # classes per token
    T = cfg.N // getattr(cfg, "group", 1)
    enc = getattr(cfg, "encoder", False)
    ent = [("tok_emb", (V if enc else V + 1, d), "w"), ("pos_emb", (T, d), "w")]
    for l in range(cfg.n_layers):
        p = f"l{l}."
        ent += [
            (p + "ln1_g", (d,), "gain"), (p + "ln1_b", (d,), "bias"),
            (p + "W_qkv", (d, 3 * d), "w"), (p + "b_qkv", (3 * d,), "bias"),
            (p + "codebook", (H, Q, d // H), "w"),
            (p + "W_o", (d, d), "w"), (p + "b_o", (d,), "bias"),
            (p + "ln2_g", (d,), "gain"), (p + "ln2_b", (d,), "bias"),
            (p + "W1", (d, F), "w"), (p + "b1", (F,), "bias"),
            (p + "W2", (F, d), "w"), (p + "b2", (d,), "bias"),
        ]
    if getattr(cfg, "attn_tail", False):
        ent += [("tail.ln_g", (d,), "gain"), ("tail.ln_b", (d,), "bias"),
                ("tail.W_qkv", (d, 3 * d), "w"),
                ("tail.b_qkv", (3 * d,), "bias"),
                ("tail.W_o", (d, d), "w"), ("tail.b_o", (d,), "bias")]
    ent += [("lnf_g", (d,), "gain"), ("lnf_b", (d,), "bias"),
            ("W_head", (d, 1 if enc else V), "w"),
            ("b_head", (1 if enc else V,), "bias")]
    out, off = [], 0
    for name, shape, kind in ent:
        n = 1
        for s in shape:
            n *= s
        out.append((name, shape, kind, off, n))
        off += n
    return out


def param_count(cfg) -> int:
    lay = param_layout(cfg)
    return lay[-1][3] + lay[-1][4]
