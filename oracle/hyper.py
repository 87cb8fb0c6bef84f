"""Model hyper-parameters and the B2 packing order (oracle side).

Readings fixed here (the paper gives only "radial functions", "spherical harmonics"
and the descriptor sizes 420 / 112, Section V.B):
  * species are indexed by atomic number order (H = 0, Pt = 1);
  * n_rad radial functions n = 0..n_rad-1 and angular channels l = 0..l_max;
  * a radial channel is a = s * n_rad + n;
  * B2 keeps every unordered channel pair a <= b (diagonal included) once, without
    extra weights, for each l. With two species, n_rad = 7, l_max = 3 this gives the
    paper's 420 components and 112 for one species (Section V.B); n_rad = 8 gives 544
    and 144;
  * packing: species-pair blocks (s1 <= s2) in order, inside a block the radial pairs
    (n_a, n_b) row-major (n_a <= n_b when s1 == s2), l fastest. A single-species block
    is therefore contiguous: the first 144 components for H only, the last 144 for Pt.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Hyper:
    n_species: int = 2
    n_rad: int = 8
    l_max: int = 3
    r_cut: float = 4.5

    @property
    def n_channels(self) -> int:
        return self.n_species * self.n_rad

    @property
    def n_lm(self) -> int:
        return (self.l_max + 1) ** 2

    def pairs(self):
        """Channel pairs (a, b) in packing order (l not included)."""
        out = []
        s_n = self.n_species
        for s1 in range(s_n):
            for s2 in range(s1, s_n):
                for na in range(self.n_rad):
                    for nb in range(self.n_rad):
                        if s1 == s2 and nb < na:
                            continue
                        out.append((s1 * self.n_rad + na, s2 * self.n_rad + nb))
        return out

    @property
    def n_desc(self) -> int:
        return len(self.pairs()) * (self.l_max + 1)

    def block_slice(self, s1: int, s2: int) -> slice:
        """Slice of the packed descriptor holding the (s1, s2) species-pair block."""
        start = 0
        for a in range(self.n_species):
            for b in range(a, self.n_species):
                size = (self.n_rad * (self.n_rad + 1) // 2 if a == b else self.n_rad * self.n_rad) * (self.l_max + 1)
                if (a, b) == (min(s1, s2), max(s1, s2)):
                    return slice(start, start + size)
                start += size
        raise ValueError((s1, s2))


DEFAULT = Hyper()
