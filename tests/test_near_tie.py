"""CPU checks of the near-tie rule the GPU parity tests apply
(tests/near_tie.py): a code difference caused by a small perturbation of
the quantizer's input at a near-tie is explained; a wrong code, or a
perturbation larger than the other rows', is not."""
import numpy as np

from near_tie import explain
from oracle import network as net


def _setup(seed=0, N=12, d=8, Q=5, H=2, nl=2):
    rng = np.random.default_rng(seed)
    cbs = [rng.standard_normal((H, Q, d // H)) for _ in range(nl)]
    a = rng.standard_normal((nl, N, d))
    codes = np.stack([net.quantize(a[l], cbs[l])[0] for l in range(nl)])
    return rng, cbs, a, codes


def test_identical_codes_give_none():
    _, cbs, a, codes = _setup()
    assert explain(cbs, codes, a, codes, a) is None


def test_small_perturbation_at_a_near_tie_is_explained():
    rng, cbs, a, codes = _setup(1)
    l, i, h = 0, 5, 1
    m = cbs[l].shape[2]
    w0 = cbs[l][h, 0]
    w1 = cbs[l][h, 1]
    # put row i of head h exactly between codewords 0 and 1, nudged to 0
    mid = 0.5 * (w0 + w1)
    a_o = a.copy()
    a_o[l, i, h * m:(h + 1) * m] = mid + 1e-9 * (w0 - w1)
    # keep both codewords the nearest two
    cbs[l][h, 2:] += 50.0
    c_o = np.stack([net.quantize(a_o[k], cbs[k])[0] for k in range(2)])
    assert c_o[l, i, h] == 0
    # the "GPU" sees every row perturbed by ~1e-7 relative, this one to 1
    a_g = a_o * (1 + 1e-7 * rng.standard_normal(a_o.shape))
    a_g[l, i, h * m:(h + 1) * m] = mid - 1e-9 * (w0 - w1)
    c_g = c_o.copy()
    c_g[l, i, h] = 1
    # only layer l differs (later layers would follow from the flip)
    ex = explain(cbs, c_g, a_g, c_o, a_o)
    assert ex["layer"] == l and len(ex["flips"]) == 1
    assert ex["ok"], ex


def test_wrong_code_is_not_explained():
    rng, cbs, a, codes = _setup(2)
    c_g = codes.copy()
    l, i, h = 1, 3, 0
    Q = cbs[l].shape[1]
    c_g[l, i, h] = (codes[l, i, h] + 1) % Q      # not the nearest codeword
    a_g = a * (1 + 1e-7 * rng.standard_normal(a.shape))
    ex = explain(cbs, c_g, a_g, codes, a)
    assert ex["layer"] == l and not ex["ok"]


def test_perturbation_beyond_the_other_rows_is_not_explained():
    rng, cbs, a, codes = _setup(3)
    l, i, h = 0, 7, 0
    m = cbs[l].shape[2]
    a_g = a * (1 + 1e-7 * rng.standard_normal(a.shape))
    # move this row's input far enough to change its code honestly
    seg = slice(h * m, (h + 1) * m)
    a_g[l, i, seg] = cbs[l][h, (codes[l, i, h] + 1) % cbs[l].shape[1]]
    c_g = codes.copy()
    c_g[l] = net.quantize(a_g[l], cbs[l])[0]
    assert c_g[l, i, h] != codes[l, i, h]
    ex = explain(cbs, c_g, a_g, codes, a)
    assert ex["layer"] == l and not ex["ok"]
