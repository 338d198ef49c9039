"""Validity of quantizer codes that differ between the GPU and the oracle.

A code is an integer decided by comparing floating-point distances (the
nearest codeword of eq. 5).  The oracle decides in FP64 at its own
attention output a_o; the GPU decides at its own attention output a_g,
which carries the rounding of its precision.  A differing code at the first
layer where the two sequences of codes part is explained -- both are
correct answers to the question each side was asked -- when

  (i)   the GPU's code is the nearest codeword to a_g up to the kernel's
        score-evaluation error: with S(c) = ||a_g - w_c||^2 in exact FP64,
        S(c_gpu) - S(c_oracle) <= eps, and
  (ii)  a_g is no further from a_o than the attention outputs of the rows
        whose codes agree: ||a_g - a_o|| / ||a_o|| of the row is at most the
        largest such relative error among the agreeing rows of that layer
        (the measured attention-output error), and
  (iii) the oracle's own gap is within what that measured error can move:
        S_o(c_gpu) - S_o(c_oracle) <= 2 ||a_g - a_o|| ||w_gpu - w_oracle||
        + eps (the score difference of two codes is affine in a with
        gradient -2 (w_gpu - w_oracle)).

eps bounds the kernel's error in the difference of two scores
||w||^2 - 2 a.w.  The BF16 mode splits a into two bfloat16 parts
(residual <= 2^-16 |a| per element), accumulates 2 x (segment width)
products in FP32 (<= 2^-15 ||a|| ||w|| for widths up to 256, doubled by the
factor 2 of the score) and takes ||w||^2 from FP32 sums of bfloat16
squares (<= 2^-16 ||w||^2); the FP32 mode's plain FP32 sums stay below the
same figures.  Per code that is at most 2^-13 ||a|| ||w|| + 2^-16 ||w||^2,
and eps is that sum over the two codes.

Test infrastructure: used by the GPU parity tests only.
"""
import numpy as np


def score_eps(a, wg, wo):
    na = np.linalg.norm(a)
    out = 0.0
    for w in (wg, wo):
        nw = np.linalg.norm(w)
        out += 2.0 ** -13 * na * nw + 2.0 ** -16 * nw * nw
    return out


def first_diff_layer(gpu_codes, oracle_codes):
    """First layer index whose codes differ ([nl][N][H] arrays), or None."""
    diff = np.asarray(gpu_codes) != np.asarray(oracle_codes)
    lay = np.nonzero(diff.any(axis=(1, 2)))[0]
    return None if len(lay) == 0 else int(lay[0])


def explain(codebooks, gpu_codes, gpu_attn, oracle_codes, oracle_attn):
    """Checks the first differing layer of one sequence.

    codebooks: per layer [H][Q][m] (the parameters both sides use);
    gpu_codes / oracle_codes: [nl][N][H]; gpu_attn / oracle_attn:
    [nl][N][d].  Returns None when every code agrees, else a dict with the
    layer, one record per differing (row, head) and ``ok`` (all explained).
    """
    l = first_diff_layer(gpu_codes, oracle_codes)
    if l is None:
        return None
    gc = np.asarray(gpu_codes[l])
    oc = np.asarray(oracle_codes[l])
    ag = np.asarray(gpu_attn[l], dtype=np.float64)
    ao = np.asarray(oracle_attn[l], dtype=np.float64)
    cb = np.asarray(codebooks[l], dtype=np.float64)
    H, Q, m = cb.shape
    # measured attention-output error of the rows whose codes agree
    agree = ~(gc != oc).any(axis=1)
    rel_rows = []
    for h in range(H):
        seg = slice(h * m, (h + 1) * m)
        num = np.linalg.norm(ag[:, seg] - ao[:, seg], axis=1)
        den = np.maximum(np.linalg.norm(ao[:, seg], axis=1), 1e-300)
        rel_rows.append(num / den)
    rel_rows = np.stack(rel_rows, axis=1)                  # [N][H]
    a_err_max = float(rel_rows[agree].max()) if agree.any() else 0.0
    recs = []
    for i, h in zip(*np.nonzero(gc != oc)):
        seg = slice(h * m, (h + 1) * m)
        wg, wo = cb[h, gc[i, h]], cb[h, oc[i, h]]
        a_g, a_o = ag[i, seg], ao[i, seg]
        eps = score_eps(a_g, wg, wo)
        gpu_gap = np.sum((a_g - wg) ** 2) - np.sum((a_g - wo) ** 2)
        orc_gap = np.sum((a_o - wg) ** 2) - np.sum((a_o - wo) ** 2)
        dlt = np.linalg.norm(a_g - a_o)
        thr = 2.0 * dlt * np.linalg.norm(wg - wo) + eps
        rec = dict(row=int(i), head=int(h), gpu_code=int(gc[i, h]),
                   oracle_code=int(oc[i, h]), gpu_gap=float(gpu_gap),
                   eps=float(eps), oracle_gap=float(orc_gap),
                   threshold=float(thr), a_rel_err=float(rel_rows[i, h]),
                   a_rel_err_agreeing_max=a_err_max)
        rec["ok"] = bool(gpu_gap <= eps and orc_gap <= thr
                         and rel_rows[i, h] <= a_err_max)
        recs.append(rec)
    return dict(layer=l, flips=recs, ok=all(r["ok"] for r in recs))
