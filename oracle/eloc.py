"""Local energy, eq. (2): E_loc(s) = sum_s' H_{s,s'} psi(s') / psi(s).

For the Marshall-rotated Heisenberg model (Sec. 4) a row of H has the
diagonal (J/4) sum_<ij> s_i s_j and, for every anti-aligned bond, the
exchanged configuration with element -J/2 (see ``lattice``).  Hence

    E_loc(s) = (J/4) sum_b s_i s_j  -  (J/2) sum_{b anti} exp(log psi(s^b) - log psi(s)).

``eloc_naive`` is that definition written out: psi is re-evaluated from
scratch on every neighbour.  ``eloc_dedup`` follows the redundancy-removal
scheme of Sec. 3.2 for the same quantized network and must agree with it.
"""
import numpy as np

from . import lattice
from . import network as net


def eloc_naive(logpsi, spins, L, periodic=True, J=1.0, marshall=True,
               return_ratios=False):
    """Local energies of spins [B, N] for any batched log-psi callable."""
    spins = np.atleast_2d(spins)
    bl = lattice.bonds(L, periodic)
    diag = lattice.diagonal(spins, bl, J)
    h_off = lattice.offdiag_element(J, marshall)
    # Gather s and all its exchanged neighbours, evaluate psi on all of them
    # in one batched call, then assemble each row of H psi / psi.
    seqs, owner = [], []
    for b in range(spins.shape[0]):
        seqs.append(spins[b])
        owner.append((b, -1))
        for _, p1, p2 in lattice.neighbours(spins[b], bl):
            seqs.append(lattice.swap(spins[b], p1, p2))
            owner.append((b, 0))
    lps = logpsi(np.stack(seqs))
    E = np.empty(spins.shape[0], dtype=np.result_type(lps, np.float64))
    ratios = []
    pos = 0
    for b in range(spins.shape[0]):
        lp0 = lps[pos]
        end = pos + 1
        while end < len(owner) and owner[end][1] == 0:
            end += 1
        r = np.exp(lps[pos + 1:end] - lp0)
        acc = 0.0
        for val in r:                       # canonical bond order
            acc += val
        E[b] = diag[b] + h_off * acc
        ratios.append(r)
        pos = end
    return (E, ratios) if return_ratios else E


def eloc_network_naive(cfg, theta, spins, return_ratios=False):
    P = net.unpack(cfg, theta)
    return eloc_naive(net.logpsi_fn(cfg, P), spins, cfg.L, cfg.periodic,
                      cfg.J, cfg.marshall, return_ratios)


def changed_inputs(u_base, u_new):
    return [int(i) for i in np.nonzero(u_base != u_new)[0]]


def eloc_dedup(cfg, theta, spins, certified=False, return_info=False):
    """Code-diff deduplicated local energy (Sec. 3.2).

    For one sample s the full network is evaluated once and its per-layer
    values are kept.  For each neighbour s' only
      * the rows whose block input differs (set C_{l-1}) get LN1/QKV again,
      * the rows at or after the first changed input (all others see an
        identical causal prefix) get attention and the quantizer again,
      * C_l = C_{l-1} plus the rows whose code changed; those rows get the
        output projection, residual and MLP again,
    and the head is re-applied to C_L and to the two exchanged sites (whose
    targets change).  A model with an attention-only half-block (no
    quantizer) after the blocks recomputes its LN + QKV on C_L and its
    attention and output projection on every row from the first changed
    input, which the head then re-reads.  With ``certified`` a row keeps s's code without a
    codebook search when the change of its attention output is smaller than
    half the gap between its best and second-best code distances (triangle
    inequality), less a small floating-point allowance.
    """
    P = net.unpack(cfg, theta)
    spins = np.atleast_2d(spins)
    K, N, d = net.group(cfg), net.n_tokens(cfg), cfg.d_model
    enc = net.encoder(cfg)
    H = cfg.vq_heads
    m = d // H
    bl = lattice.bonds(cfg.L, cfg.periodic)
    diag = lattice.diagonal(spins, bl, cfg.J)
    h_off = lattice.offdiag_element(cfg.J, cfg.marshall)
    E = np.empty(spins.shape[0])
    info = dict(ratios=[], changed=[], att_rows=[], vq_rows=[], codes=[])
    for b in range(spins.shape[0]):
        base = net.forward(cfg, P, spins[b:b + 1], keep=True)
        t0, u0 = net.tokens(spins[b:b + 1], K)
        if enc:
            u0 = t0                    # the encoder reads the tokens
        C_base = [{k: v[0] for k, v in c.items()} for c in base["caches"]]
        lp0 = None if enc else base["lp"][0]
        ell0 = None if enc else base["ell"][0]
        acc = 0.0
        for _, p1, p2 in lattice.neighbours(spins[b], bl):
            s1 = lattice.swap(spins[b], p1, p2)
            t1, u1 = net.tokens(s1[None], K)
            t1, u1 = t1[0], u1[0]
            if enc:
                u1 = t1
            C = changed_inputs(u0[0], u1)
            # tokens of the exchanged sites (one token when both fall in it)
            tp1, tp2 = p1 // K, p2 // K
            # the decoder's rows before the first changed input see an
            # unchanged prefix; every encoder row attends to the change
            pmin = 0 if enc else tp1 + 1
            xo = {i: P["tok"][u1[i]] + P["pos"][i] for i in C}
            sizes, arows, vrows, codes_sp = [len(C)], 0, 0, []
            for l, lay in enumerate(P["layers"]):
                cb = C_base[l]
                q, k, v = cb["q"].copy(), cb["k"].copy(), cb["v"].copy()
                if C:
                    rows = np.array(sorted(C))
                    qkv = net.qkv_rows(lay, np.stack([xo[i] for i in rows]))
                    q[rows], k[rows], v[rows] = (qkv[:, :d], qkv[:, d:2 * d],
                                                 qkv[:, 2 * d:])
                att = np.arange(pmin, N)
                arows += len(att)
                a = net.causal_attention(q[att], k, v, cfg.n_heads, rows=att,
                                         causal=not enc)
                codes = cb["codes"].copy()
                search = np.ones(len(att), dtype=bool)
                if certified:
                    ok = np.ones(len(att), dtype=bool)
                    for h in range(H):
                        dl = a[:, h * m:(h + 1) * m] - cb["a"][att, h * m:(h + 1) * m]
                        nd = np.sqrt((dl * dl).sum(axis=1))
                        d1, d2 = cb["d1"][att, h], cb["d2"][att, h]
                        slack = 1e-9 * (1.0 + d2)
                        ok &= nd < 0.5 * (d2 - d1) - slack
                    search = ~ok
                if search.any():
                    c_new, _, _, _ = net.quantize(a[search], lay["codebook"])
                    codes[att[search]] = c_new
                vrows += int(search.sum())
                diffrows = att[(codes[att] != cb["codes"][att]).any(axis=1)]
                C_new = sorted(set(C) | set(int(i) for i in diffrows))
                if C_new:
                    rows = np.array(C_new)
                    xin = np.stack([xo[i] if i in xo else cb["x"][i]
                                    for i in rows])
                    z = np.concatenate(
                        [lay["codebook"][h][codes[rows, h]] for h in range(H)],
                        axis=1)
                    xn = net.post_vq_rows(lay, xin, z)
                    xo = {int(i): xn[j] for j, i in enumerate(rows)}
                C = C_new
                sizes.append(len(C))
                codes_sp.append(codes)
            if "tail" in P:
                # attention-only half-block: no quantizer, so every row at
                # or after the first changed input changes; LN + QKV on the
                # rows of C_L, attention and the output projection on all
                # rows from p_min
                T, tc = P["tail"], base["tail"]
                q, k, v = tc["q"][0].copy(), tc["k"][0].copy(), tc["v"][0].copy()
                if C:
                    rows = np.array(C)
                    qkv = net.qkv_rows(dict(ln1_g=T["ln_g"], ln1_b=T["ln_b"],
                                            W_qkv=T["W_qkv"],
                                            b_qkv=T["b_qkv"]),
                                       np.stack([xo[i] for i in rows]))
                    q[rows], k[rows], v[rows] = (qkv[:, :d], qkv[:, d:2 * d],
                                                 qkv[:, 2 * d:])
                att = np.arange(pmin, N)
                arows += len(att)
                a = net.causal_attention(q[att], k, v, cfg.n_heads, rows=att)
                xin = np.stack([xo[i] if i in xo else tc["x"][0][i]
                                for i in att])
                xn = xin + a @ T["W_o"] + T["b_o"]
                xo = {int(i): xn[j] for j, i in enumerate(att)}
                C = [int(i) for i in att]
            if enc:
                # encoder head: the pooled mean changes by the rows of C_L
                c0 = base["terms"][0]
                delta = 0.0
                if C:
                    rows = np.array(C)
                    cn = net.pooled_terms(P, np.stack([xo[i] for i in rows]))
                    for j, i in enumerate(rows):
                        delta += cn[j] - c0[i]
                r = np.exp(delta / N)
                acc += r
                info["ratios"].append((b, r))
                info["changed"].append(sizes)
                info["att_rows"].append(arows)
                info["vq_rows"].append(vrows)
                info["codes"].append(np.stack(codes_sp) if codes_sp else None)
                continue
            # Head: rows of C_L get new log-probs; the tokens of the
            # exchanged sites keep s's hidden state but change target.
            delta = 0.0
            head_rows = sorted(set(C) | {tp1, tp2})
            lpn = {}
            if C:
                rows = np.array(C)
                lpr = net.head_logprobs(P, np.stack([xo[i] for i in rows]))
                lpn = {int(i): lpr[j] for j, i in enumerate(rows)}
            for i in head_rows:
                new = lpn[i][t1[i]] if i in lpn else lp0[i][t1[i]]
                delta += new - ell0[i]
            r = np.exp(0.5 * delta)
            acc += r
            info["ratios"].append((b, r))
            info["changed"].append(sizes)
            info["att_rows"].append(arows)
            info["vq_rows"].append(vrows)
            info["codes"].append(np.stack(codes_sp) if codes_sp else None)
        E[b] = diag[b] + h_off * acc
    return (E, info) if return_info else E


def batch_stats(E, logpsi=None):
    """Plain batch mean and (biased) variance of E_loc; with log psi given,
    also the psi^2-weighted mean (log-sum-exp weights)."""
    E = np.asarray(E, dtype=np.float64)
    out = dict(mean=E.mean(), var=E.var())
    if logpsi is not None:
        w = 2.0 * np.asarray(logpsi)
        w = np.exp(w - w.max())
        out["weighted_mean"] = float((w * E).sum() / w.sum())
    return out
