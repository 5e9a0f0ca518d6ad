"""Seeded synthetic inputs for the AO -> MO value/gradient/Laplacian path.

This module only draws numbers: geometries, raw basis-set parameters
(exponents and contraction coefficients, never normalisation factors),
MO coefficients, electron coordinates and adjoint weights.  It holds none of
the method's arithmetic, so both the FP64 CPU oracle and the GPU library can
consume the same inputs while deriving everything else on their own.

The paper's benchmark systems (a Cu(II)-peptide complex in cc-pVDZ, C60 in
cc-pVQZ, aspirin, polyenes; Section 3.1, 3.2 and Section 4) and their basis
sets are not available, so these seeded stand-ins replace them.  They keep the
structure of real all-electron Gaussian bases: one basis per element, shells
of contracted Cartesian Gaussians with 1-6 primitives whose exponents span
0.1 .. 1e4 bohr^-2 (the range of tight core to diffuse valence primitives),
carbon and hydrogen atoms at realistic densities, electrons clustered around
the nuclei.

Draw order (fixed, so that a seed always reproduces the same system):
``SeedSequence(seed).spawn(5)`` gives independent streams for
geometry, basis, MO coefficients, electrons and adjoint weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Cartesian function counts per angular momentum l: (l+1)(l+2)/2.
N_CART = {0: 1, 1: 3, 2: 6, 3: 10}

# Shell recipes: angular momentum of each shell of an element's basis.
RECIPE_HEAVY_SMALL = (0, 0, 0, 1, 1, 2)                    # 3s2p1d -> 15 AOs
RECIPE_H_SMALL = (0, 0, 1)                                 # 2s1p   ->  5 AOs
RECIPE_HEAVY_LARGE = (0, 0, 0, 0, 1, 1, 1, 2, 2, 3)        # 4s3p2d1f -> 35 AOs
RECIPE_H_LARGE = (0, 0, 0, 1, 1, 2)                        # 3s2p1d -> 15 AOs
RECIPE_TM_DZ = (0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 3)  # 6s5p3d1f -> 49 AOs


@dataclass
class System:
    """One molecule plus a batch of walkers.

    Arrays follow the library's C-ABI conventions (bohr, C order):
      nucl_coord        [nucl, 3]  float64
      nucl_charge       [nucl]     int32 (electrons placed around each nucleus)
      shell_nucleus     [shell]    int64
      shell_ang_mom     [shell]    int32 (0..3)
      shell_prim_offset [shell+1]  int64 (primitives of shell s are
                                         offset[s] .. offset[s+1]-1)
      exponent          [prim]     float64 (gamma)
      coefficient       [prim]     float64 (raw contraction coefficient a)
      mo_coef           [mo, ao]   float64
      elec_coord        [walk, elec, 3] float64
    """
    name: str
    nucl_coord: np.ndarray
    nucl_charge: np.ndarray
    shell_nucleus: np.ndarray
    shell_ang_mom: np.ndarray
    shell_prim_offset: np.ndarray
    exponent: np.ndarray
    coefficient: np.ndarray
    mo_coef: np.ndarray
    elec_coord: np.ndarray
    seed: int = 0
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def nucl_num(self) -> int:
        return int(self.nucl_coord.shape[0])

    @property
    def shell_num(self) -> int:
        return int(self.shell_ang_mom.shape[0])

    @property
    def prim_num(self) -> int:
        return int(self.exponent.shape[0])

    @property
    def ao_num(self) -> int:
        return int(sum(N_CART[int(l)] for l in self.shell_ang_mom))

    @property
    def mo_num(self) -> int:
        return int(self.mo_coef.shape[0])

    @property
    def walk_num(self) -> int:
        return int(self.elec_coord.shape[0])

    @property
    def elec_num(self) -> int:
        return int(self.elec_coord.shape[1])

    @property
    def point_num(self) -> int:
        return self.walk_num * self.elec_num

    def points(self) -> np.ndarray:
        """Electron coordinates flattened to [walk*elec, 3]."""
        return np.ascontiguousarray(self.elec_coord.reshape(-1, 3))

    def with_walkers(self, walkers: int) -> "System":
        """Same molecule with only the first `walkers` walkers."""
        s = System(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        s.elec_coord = np.ascontiguousarray(self.elec_coord[:walkers])
        return s


def _streams(seed: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(5)]


def _draw_shell(rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """1..6 primitives, log10(gamma) ~ U(-1, 4), a ~ U(0.1, 1), ascending gamma."""
    n = int(rng.integers(1, 7))
    gam = 10.0 ** rng.uniform(-1.0, 4.0, size=n)
    a = rng.uniform(0.1, 1.0, size=n)
    order = np.argsort(gam, kind="stable")
    return gam[order], a[order]


def _draw_element_basis(rng: np.random.Generator, recipe: Sequence[int]):
    return [(int(l),) + _draw_shell(rng) for l in recipe]


def _assemble(name, coords, charges, elem_of_atom, bases, rng_c, rng_e,
              n_mo, walkers, seed, meta) -> System:
    sh_nuc, sh_l, offs, gam, coef = [], [], [0], [], []
    for a, el in enumerate(elem_of_atom):
        for (l, g, c) in bases[el]:
            sh_nuc.append(a)
            sh_l.append(l)
            gam.append(g)
            coef.append(c)
            offs.append(offs[-1] + len(g))
    ao_num = int(sum(N_CART[l] for l in sh_l))
    mo = rng_c.normal(0.0, 1.0 / np.sqrt(ao_num), size=(n_mo, ao_num))
    # Z_A electrons per nucleus at R_A + N(0, I_3); walkers independent.
    centres = np.repeat(coords, charges, axis=0)
    elec = centres[None, :, :] + rng_e.normal(0.0, 1.0, size=(walkers, centres.shape[0], 3))
    return System(
        name=name,
        nucl_coord=np.ascontiguousarray(coords, dtype=np.float64),
        nucl_charge=np.asarray(charges, dtype=np.int32),
        shell_nucleus=np.asarray(sh_nuc, dtype=np.int64),
        shell_ang_mom=np.asarray(sh_l, dtype=np.int32),
        shell_prim_offset=np.asarray(offs, dtype=np.int64),
        exponent=np.concatenate(gam).astype(np.float64),
        coefficient=np.concatenate(coef).astype(np.float64),
        mo_coef=np.ascontiguousarray(mo, dtype=np.float64),
        elec_coord=np.ascontiguousarray(elec, dtype=np.float64),
        seed=seed,
        meta=meta,
    )


def _pack_atoms(rng: np.random.Generator, n: int, box: float, min_sep: float) -> np.ndarray:
    """Rejection-sample n points uniform in [0, box)^3 with pairwise distance >= min_sep."""
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 200000 * max(n, 1):
            raise RuntimeError("could not place atoms")
        p = rng.uniform(0.0, box, size=3)
        if k == 0 or np.min(np.sum((pts[:k] - p) ** 2, axis=1)) >= min_sep * min_sep:
            pts[k] = p
            k += 1
    return pts


def water_like(walkers: int = 128, seed: int = 0) -> System:
    """Z=8 nucleus at the origin and two H at 1.8 bohr with a random angle in
    (pi/3, pi); heavy 3s2p1d + H 2s1p Cartesian basis (25 AOs); 25 MOs with
    C ~ N(0, 1/25); 10 electrons; `walkers` walkers."""
    rg, rb, rc, re, _ = _streams(seed)
    th = rg.uniform(np.pi / 3, np.pi)
    coords = np.array([[0.0, 0.0, 0.0], [1.8, 0.0, 0.0], [1.8 * np.cos(th), 1.8 * np.sin(th), 0.0]])
    bases = {"O": _draw_element_basis(rb, RECIPE_HEAVY_SMALL), "H": _draw_element_basis(rb, RECIPE_H_SMALL)}
    return _assemble("water_like", coords, [8, 1, 1], ["O", "H", "H"], bases, rc, re,
                     25, walkers, seed, {"box": None})


def ch_cluster(n_c: int, n_h: int, box: float, walkers: int, seed: int,
               heavy=RECIPE_HEAVY_SMALL, light=RECIPE_H_SMALL, n_mo: Optional[int] = None,
               name: str = "ch_cluster") -> System:
    """n_c carbons (Z=6) then n_h hydrogens uniform in a `box`-bohr cube with
    1.5-bohr minimum separation; one basis per element; n_mo MOs (default
    ao_num/2) with C ~ N(0, 1/ao_num); Z_A electrons per nucleus."""
    rg, rb, rc, re, _ = _streams(seed)
    coords = _pack_atoms(rg, n_c + n_h, box, 1.5)
    bases = {"C": _draw_element_basis(rb, heavy), "H": _draw_element_basis(rb, light)}
    elems = ["C"] * n_c + ["H"] * n_h
    charges = [6] * n_c + [1] * n_h
    ao = n_c * sum(N_CART[l] for l in heavy) + n_h * sum(N_CART[l] for l in light)
    if n_mo is None:
        n_mo = max(ao // 2, 1)
    return _assemble(name, coords, charges, elems, bases, rc, re, n_mo, walkers, seed,
                     {"box": box, "n_c": n_c, "n_h": n_h})


def medium(walkers: int = 512, seed: int = 0) -> System:
    """40 C + 40 H in a 20-bohr cube, 800 AOs, 400 MOs, 280 electrons."""
    return ch_cluster(40, 40, 20.0, walkers, seed, n_mo=400, name="ch80_800ao")


def large(walkers: int = 64, seed: int = 0) -> System:
    """150 C + 150 H in a 35-bohr cube, heavy 4s3p2d1f + H 3s2p1d -> 7500 AOs,
    1050 MOs, 1050 electrons."""
    return ch_cluster(150, 150, 35.0, walkers, seed, heavy=RECIPE_HEAVY_LARGE,
                      light=RECIPE_H_LARGE, n_mo=1050, name="ch300_7500ao")


def peptide_like(grid_n: int = 100, seed: int = 0, margin: float = 4.0) -> System:
    """Stand-in for the density benchmark of Section 5.4 (a Cu(II)-peptide
    complex, C34 H48 Cu N11 O10, in cc-pVDZ: 1114 AOs, 218 occupied MOs, on a
    100^3 grid).  34 C, 11 N, 10 O (3s2p1d each), 48 H (2s1p) and one Cu
    (6s5p3d1f), each element with its own drawn basis -> 1114 Cartesian AOs;
    atoms uniform in a cube at the medium system's atom density (80 atoms per
    20^3 bohr^3) with 1.5-bohr minimum separation; 1053 MOs with
    C ~ N(0, 1/1114), of which the first 218 are doubly occupied
    (meta["occ"]).  The points are a grid_n^3 Cartesian grid over the atoms'
    cube plus `margin` bohr on every side (z fastest, as in a cube file),
    held as one walker of grid_n^3 "electrons"."""
    rg, rb, rc, re, _ = _streams(seed)
    elems = ["C"] * 34 + ["N"] * 11 + ["O"] * 10 + ["H"] * 48 + ["Cu"]
    charges = {"C": 6, "N": 7, "O": 8, "H": 1, "Cu": 29}
    n_at = len(elems)
    box = 20.0 * (n_at / 80.0) ** (1.0 / 3.0)
    coords = _pack_atoms(rg, n_at, box, 1.5)
    bases = {"C": _draw_element_basis(rb, RECIPE_HEAVY_SMALL),
             "N": _draw_element_basis(rb, RECIPE_HEAVY_SMALL),
             "O": _draw_element_basis(rb, RECIPE_HEAVY_SMALL),
             "H": _draw_element_basis(rb, RECIPE_H_SMALL),
             "Cu": _draw_element_basis(rb, RECIPE_TM_DZ)}
    s = _assemble("peptide_like", coords, [charges[e] for e in elems], elems, bases, rc, re,
                  1053, 1, seed, {"box": box})
    ax = np.linspace(-margin, box + margin, grid_n)
    gx, gy, gz = np.meshgrid(ax, ax, ax, indexing="ij")
    grid = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    s.elec_coord = np.ascontiguousarray(grid.reshape(1, -1, 3))
    occ = np.zeros(s.mo_num)
    occ[:218] = 2.0
    s.meta = dict(s.meta, occ=occ, grid_n=grid_n, spacing=float(ax[1] - ax[0]))
    return s


def molecule_batch(n_mol: int = 96, seed: int = 0) -> List[System]:
    """`n_mol` molecules with atom count uniform in 4..60 (ceil(n/2) C,
    floor(n/2) H) and walkers uniform in 8..128; molecule m uses child seed m
    of the batch seed.  Atom density equals the medium system's
    (80 atoms per 20^3 bohr^3); basis recipe 3s2p1d / 2s1p; MOs = AOs/2."""
    top = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    n_atoms = top.integers(4, 61, size=n_mol)
    walkers = top.integers(8, 129, size=n_mol)
    kids = np.random.SeedSequence(seed + 1).spawn(n_mol)
    out = []
    for m in range(n_mol):
        n = int(n_atoms[m])
        n_c, n_h = (n + 1) // 2, n // 2
        box = 20.0 * (n / 80.0) ** (1.0 / 3.0)
        child = int(kids[m].generate_state(1)[0])
        out.append(ch_cluster(n_c, n_h, box, int(walkers[m]), child, name=f"mol{m}"))
    return out


def adjoint_weights(sys_: System, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """W ~ N(0, 1) of shape [walk, elec, 5, mo] (the loss is sum(W * mo_vgl))."""
    rw = _streams(seed)[4]
    return rw.standard_normal((sys_.walk_num, sys_.elec_num, 5, sys_.mo_num)).astype(dtype)


def tiny_system(ls: Sequence[int], n_prim: int = 2, seed: int = 0, walkers: int = 1,
                elec: int = 4, gamma_range=(-0.5, 1.0), n_nuc: int = 2) -> System:
    """Small hand-sized system for pins: `n_nuc` nuclei sharing a basis with
    shells of angular momenta `ls`, exponents log10-uniform in `gamma_range`."""
    rg, rb, rc, re, _ = _streams(seed)
    coords = rg.uniform(-1.0, 1.0, size=(n_nuc, 3))
    shells = []
    for l in ls:
        g = np.sort(10.0 ** rb.uniform(gamma_range[0], gamma_range[1], size=n_prim))
        shells.append((int(l), g, rb.uniform(0.1, 1.0, size=n_prim)))
    bases = {"X": shells}
    charges = [elec // n_nuc + (1 if i < elec % n_nuc else 0) for i in range(n_nuc)]
    ao = n_nuc * sum(N_CART[l] for l in ls)
    return _assemble("tiny", coords, charges, ["X"] * n_nuc, bases, rc, re, ao, walkers,
                     seed, {})


CONFIGS = {
    "water_like": water_like,
    "medium": medium,
    "large": large,
    "peptide_like": peptide_like,
}
