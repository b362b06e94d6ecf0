"""Per-object NeRF architecture alpha (Sec. III: a hash-grid encoding plus a
shallow MLP whose hyper-parameters are searched per category in Sec. III-A).

Level resolutions follow the multiresolution hash encoding of Mueller et al.
(2022): N_l = floor(N_min * b**l).  They are computed here once, in exact
rational arithmetic, and handed to both the oracle and the GPU library as
integers, so neither side depends on a floating-point pow().
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import Tuple

N_OUT = 4  # sigma + RGB head


def level_resolutions(n_levels: int, base_res: int, growth: str | float) -> Tuple[int, ...]:
    b = Fraction(str(growth))
    out = []
    for l in range(n_levels):
        v = Fraction(base_res) * b**l
        out.append(v.numerator // v.denominator)
    return tuple(out)


@dataclass(frozen=True)
class Arch:
    n_levels: int = 16
    log2_table: int = 19
    n_features: int = 2
    base_res: int = 16
    growth: str = "1.5"
    width: int = 64
    hidden: int = 2
    resolutions: Tuple[int, ...] = field(default=())
    mlp_dtype: str = "fp32"     # "fp32" | "bf16" | "fp16"
    table_dtype: str = "fp32"   # "fp32" | "fp16" (an FP16 copy read by the forward gathers)

    def __post_init__(self):
        if not self.resolutions:
            object.__setattr__(self, "resolutions",
                               level_resolutions(self.n_levels, self.base_res, self.growth))
        assert len(self.resolutions) == self.n_levels

    @property
    def table_size(self) -> int:
        return 1 << self.log2_table

    @property
    def in_dim(self) -> int:
        return self.n_levels * self.n_features

    @property
    def n_table_params(self) -> int:
        return self.n_levels * self.table_size * self.n_features

    def layer_shapes(self):
        """(out, in) of W_1 .. W_D, W_out, stored row-major in that order."""
        shapes = [(self.width, self.in_dim)]
        shapes += [(self.width, self.width)] * (self.hidden - 1)
        shapes.append((N_OUT, self.width))
        return shapes

    @property
    def n_mlp_params(self) -> int:
        return sum(o * i for o, i in self.layer_shapes())

    @property
    def n_params(self) -> int:
        return self.n_table_params + self.n_mlp_params

    def dense_levels(self):
        """Levels whose (N+1)^3 lattice fits the table 1:1."""
        return [l for l, n in enumerate(self.resolutions) if (n + 1) ** 3 <= self.table_size]


# Plain single-object step (8 levels x 2^14, 64-wide MLP with one hidden layer)
ARCH_SMALL = Arch(n_levels=8, log2_table=14, n_features=2, base_res=16, growth="1.5",
                  width=64, hidden=1)
# Prior-sampling workload (16 levels x 2^19, MLP 64 x 2 hidden)
ARCH_LARGE = Arch(n_levels=16, log2_table=19, n_features=2, base_res=16, growth="1.5",
                  width=64, hidden=2)
