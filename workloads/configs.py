"""Workload configurations (lattice + transformer shape + batch).

The five workloads mirror the paper's setting (2-D spin-1/2 Heisenberg model,
Sec. 4; autoregressive transformer with a vector quantizer after every
self-attention, Sec. 3.1) at the sizes this project measures:

  small   4x4,   d=16,  1 layer,  2 heads, MLP 64,   Q=16,   B=256,  fp64
  medium  10x10, d=64,  4 layers, 4 heads, MLP 256,  Q=256,  B=4096, fp32
  large   16x16, d=128, 8 layers, 8 heads, MLP 512,  Q=1024, B=8192, bf16
  multi   6x6..20x20 lattices, d=128, 6 layers, 8 heads, MLP 512, Q=512, bf16
  grad    20x20, d=256, 12 layers, 8 heads, MLP 1024, Q=1024, B=2048, bf16
  large_g4 the large model over tokens of 4 spins (64 tokens), B=8192, bf16
  small_g4 the small model over tokens of 4 spins (4 tokens), B=64, f64
  table1  the paper's Table 1 network (3 blocks + attention-only half-block,
          d=256, 8 heads, 64 codes) on the open 8x8 lattice, B=4096, bf16
  tfim    1-D transverse-field Ising chain of 384 sites (open, Gamma = J = 1),
          d=256, 1 layer, 8 heads, MLP 1024, 4 x 64 codes, B=2048, bf16

Lattices are periodic with J=1 in the Marshall-rotated basis unless stated.
"""
from dataclasses import dataclass, replace, asdict

PRECISIONS = ("f64", "f32", "bf16")


@dataclass(frozen=True)
class ModelConfig:
    name: str
    L: int
    d_model: int
    n_layers: int
    n_heads: int
    d_ff: int
    codebook_size: int          # Q, codes per quantizer head
    vq_heads: int = 1           # H of the multi-head quantizer
    periodic: bool = True
    marshall: bool = True
    J: float = 1.0
    precision: str = "f64"
    batch: int = 256
    spin_seed: int = 1000
    param_seed: int = 0
    hamiltonian: str = "heisenberg"   # or "tfim": chain of L sites
    gamma: float = 1.0                # transverse field of the TFIM
    attn_tail: bool = False           # attention-only half-block after the
                                      # blocks (no quantizer, no MLP)
    group: int = 1                    # spins per token (Sec. 3.1: tokens are
                                      # groups of K particles)
    encoder: bool = False             # bidirectional encoder with mean
                                      # pooling as log psi (Sec. 3.1)

    @property
    def N(self) -> int:
        return self.L if self.hamiltonian == "tfim" else self.L * self.L

    @property
    def T(self) -> int:
        """Sequence length: tokens of ``group`` consecutive sites."""
        if self.N % self.group:
            raise ValueError(f"{self.N} sites do not split into tokens of "
                             f"{self.group}")
        return self.N // self.group

    @property
    def d_head(self) -> int:
        return self.d_model // self.n_heads

    def as_dict(self):
        return asdict(self)


CONFIGS = {
    "small": ModelConfig("small", L=4, d_model=16, n_layers=1, n_heads=2,
                         d_ff=64, codebook_size=16, precision="f64",
                         batch=256, spin_seed=1001),
    "medium": ModelConfig("medium", L=10, d_model=64, n_layers=4, n_heads=4,
                          d_ff=256, codebook_size=256, precision="f32",
                          batch=4096, spin_seed=1002),
    "large": ModelConfig("large", L=16, d_model=128, n_layers=8, n_heads=8,
                         d_ff=512, codebook_size=1024, precision="bf16",
                         batch=8192, spin_seed=1003),
    "grad": ModelConfig("grad", L=20, d_model=256, n_layers=12, n_heads=8,
                        d_ff=1024, codebook_size=1024, precision="bf16",
                        batch=2048, spin_seed=1005),
}

# One-dimensional transverse-field Ising chain at the critical field
# (Gamma = J = 1, open boundaries): the paper's second workload (Sec. 4,
# Fig. 2: one block, width 256, 8 heads, a quantizer of 4 heads x 64 codes,
# up to 384 spins).  Spins are uniformly random (no Sz constraint).
CONFIGS["tfim"] = ModelConfig("tfim", L=384, d_model=256, n_layers=1,
                              n_heads=8, d_ff=1024, codebook_size=64,
                              vq_heads=4, periodic=False, marshall=False,
                              precision="bf16", batch=2048, spin_seed=1006,
                              hamiltonian="tfim", gamma=1.0)
CONFIGS["tfim_small"] = ModelConfig("tfim_small", L=10, d_model=16,
                                    n_layers=1, n_heads=2, d_ff=64,
                                    codebook_size=16, vq_heads=2,
                                    periodic=False, marshall=False,
                                    precision="f64", batch=64,
                                    spin_seed=1007, hamiltonian="tfim",
                                    gamma=1.0)

# The architecture of the paper's Table 1: three VQ transformer blocks and
# an attention-only half-block (no quantizer), width 256, 8 heads, one
# quantizer head of 64 codes (the table's 6-bit column), on the open 8x8
# lattice (Sec. 4); seeded random weights stand in for the distilled ones.
CONFIGS["table1"] = ModelConfig("table1", L=8, d_model=256, n_layers=3,
                                n_heads=8, d_ff=1024, codebook_size=64,
                                vq_heads=1, periodic=False, precision="bf16",
                                batch=4096, spin_seed=1008, attn_tail=True)

# Tokens of four spins (Sec. 3.1 groups of K particles; Sec. 3.2 uses
# groups of 4): the 16x16 model over 64 tokens of 16 values, and a 4x4
# FP64 model over 4 tokens for oracle parity.
CONFIGS["large_g4"] = replace(CONFIGS["large"], name="large_g4", group=4,
                              spin_seed=1009)
CONFIGS["small_g4"] = replace(CONFIGS["small"], name="small_g4", group=4,
                              batch=64, spin_seed=1010)

# The bidirectional encoder with mean pooling as log psi (Sec. 3.1) at the
# 16x16 model's sizes: every row attends to every position, so a neighbour
# re-attends all rows.
CONFIGS["large_enc"] = replace(CONFIGS["large"], name="large_enc", encoder=True,
                               spin_seed=1014)

# Mixed-lattice batch: one parameter buffer per lattice, uneven sample counts.
MULTI_LATTICE = tuple(
    ModelConfig(f"multi_L{L}", L=L, d_model=128, n_layers=6, n_heads=8,
                d_ff=512, codebook_size=512, precision="bf16", batch=B,
                spin_seed=1400 + k, param_seed=k)
    for k, (L, B) in enumerate([(6, 512), (8, 1024), (12, 2048), (16, 4096),
                                (20, 8192)]))


def config_by_name(name: str) -> ModelConfig:
    if name in CONFIGS:
        return CONFIGS[name]
    for c in MULTI_LATTICE:
        if c.name == name:
            return c
    raise KeyError(name)


def with_batch(cfg: ModelConfig, batch: int, **kw) -> ModelConfig:
    return replace(cfg, batch=batch, **kw)
