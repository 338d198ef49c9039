"""Pins of the transverse-field Ising oracle (oracle/tfim.py, Sec. 4).

* Exact diagonalisation of the Pauli-matrix Hamiltonian at the critical
  field (J = Gamma = 1) against the free-fermion closed forms: periodic
  chain E0 = -2 / sin(pi / (2N)), open chain E0 = 1 - 1 / sin(pi / (2(2N+1))).
* Sum rule (eqs. 1-2): the psi^2-weighted mean of E_loc over all 2^N
  configurations equals <psi|H|psi>/<psi|psi> with H from Pauli matrices,
  for a random network (open and periodic).
* Zero variance: E_loc of the exact ground state is E0 on every
  configuration.
* Constant psi: E_loc = -J sum s_i s_j - Gamma N.
A wrong sign of either term, a missing flip or a wrong bond set fails one
of these."""
from dataclasses import replace

import numpy as np
import pytest
from scipy.sparse.linalg import eigsh

from oracle import ed, tfim
from oracle import network as net
from workloads import CONFIGS, make_params


@pytest.mark.parametrize("N", [6, 8, 10])
def test_ed_matches_closed_forms_at_the_critical_field(N):
    e_p = tfim.ground_energy(N, True)
    e_o = tfim.ground_energy(N, False)
    assert abs(e_p + 2.0 / np.sin(np.pi / (2 * N))) < 1e-10
    assert abs(e_o - (1.0 - 1.0 / np.sin(np.pi / (2 * (2 * N + 1))))) < 1e-10


@pytest.mark.parametrize("periodic", [False, True])
def test_sum_rule_random_network(periodic):
    mc = replace(CONFIGS["tfim_small"], L=8, periodic=periodic)
    theta = make_params(mc, std=0.3)
    P = net.unpack(mc, theta)
    states = tfim.all_states(mc.N)
    lp = net.logpsi_fn(mc, P, chunk=256)(states)
    E = tfim.eloc_naive(net.logpsi_fn(mc, P, chunk=256), states, mc.N,
                        periodic, mc.J, mc.gamma)
    w = np.exp(2.0 * lp)
    H = tfim.hamiltonian(mc.N, periodic, mc.J, mc.gamma)
    v = np.zeros(2 ** mc.N)
    v[ed.index_of_config(states)] = np.exp(lp)
    ref = v @ (H @ v) / (v @ v)
    assert abs((w * E).sum() / w.sum() - ref) < 1e-12 * abs(ref)


def test_zero_variance_for_the_ground_state():
    N = 8
    H = tfim.hamiltonian(N, False)
    vals, vecs = eigsh(H, k=1, which="SA", tol=1e-12)
    v = vecs[:, 0] * np.sign(vecs[:, 0].sum())
    assert (v > 0).all()                     # stoquastic: positive
    lut = np.log(v)

    def logpsi(spins):
        return lut[ed.index_of_config(spins)]
    states = tfim.all_states(N)
    E = tfim.eloc_naive(logpsi, states, N, False)
    assert np.abs(E - vals[0]).max() < 1e-9


def test_constant_psi():
    N = 7
    states = tfim.all_states(N)[::5]
    E = tfim.eloc_naive(lambda s: np.zeros(s.shape[0]), states, N, True,
                        J=0.7, gamma=1.3)
    s = states.astype(float)
    ref = -0.7 * (s * np.roll(s, -1, axis=1)).sum(axis=1) - 1.3 * N
    assert np.allclose(E, ref, rtol=0, atol=1e-12)
