"""FP64 CPU oracle for the VQ-NQS local-energy path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import or call this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code with the GPU implementation: only the seeded input generators in
``workloads`` serve both.

Plain, slow, obviously-correct NumPy float64 code that follows the paper:

* ``lattice``  - nearest-neighbour bonds of the L x L lattice, the exact
  diagonal of the Heisenberg Hamiltonian and its off-diagonal (spin-exchange)
  neighbours in the Marshall-rotated basis (Sec. 2 k-local discussion; Sec. 4
  Hamiltonian and Marshall sign rule).
* ``network``  - the autoregressive transformer with a vector quantizer after
  each self-attention (Sec. 3.1, eqs. 4-6; chain-rule distribution of Sec. 2),
  log psi = 1/2 log P with zero phase (Sec. 4); tokens of one spin, or of
  groups of K spins with 2^K values (Sec. 3.1); or the bidirectional
  encoder with mean pooling as log psi (Sec. 3.1's other network).
* ``eloc``     - the local energy of eq. (2) by naive re-evaluation of psi on
  every neighbour, and the code-diff deduplicated evaluation of Sec. 3.2 as a
  cross-check with its changed-row counters.
* ``ed``       - exact diagonalisation from an independent Pauli Kronecker
  construction of the Hamiltonian (pins units, boundary conditions and sign).
* ``grad``     - reference d log psi / d theta with the straight-through
  estimator of eqs. (7)-(8), in float64 autograd on the CPU.

Pins (tests/test_oracle_*.py):
  lattice/eloc: exact-diagonalisation energies (the paper's 4x4 table entry),
    the sum rule <psi|H|psi>/<psi|psi> = Born-weighted mean of E_loc, zero
    variance for exact eigenstates, closed forms for constant psi.
  network: normalisation of the autoregressive distribution over all 2^N
    states, causal-prefix invariance, per-operation reduction to library
    routines (layer norm, causal attention, GELU, nearest-codeword search),
    head-permutation invariance.
  eloc_dedup: identical codes and equal E_loc to the naive evaluation.
  grad: central finite differences of the relaxed straight-through surrogate.
  tokens of K spins: the token of a group by hand, the closed form for
    zero weights but the head bias, normalisation over all states, the
    sampler's histogram, dedup = plain, central differences.
  encoder: the closed form for zero weights but the head bias, symmetry
    under token permutations without position embeddings, bidirectional
    attention, dedup = plain, central differences.
  whole network: closed forms from library routines where the blocks pass
    their input through (output projection and second MLP matrix at zero)
    and where every attention score is zero (query and key projections at
    zero: attention is the running mean of the values), for the decoder with
    and without the attention-only half-block, tokens of 1, 2 and 4 spins,
    and the encoder; a dropped residual, a shifted mask, LN2 on the wrong
    stream, a missing input shift or pooling before the final LN fail them.
"""
from . import lattice, network, eloc, ed  # noqa: F401
