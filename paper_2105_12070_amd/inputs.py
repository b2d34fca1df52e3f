"""Seeded synthetic chemistry workloads (mechanisms and cell states).

The paper's benchmarks use real kinetic mechanisms (GRI-3.0 with 53 species and
325 reactions, Yao with 54/269, DRM19 with 21/83; section 3) and CFD fields.
Neither is available here, so every workload is synthetic: a random but
element-balanced mechanism in Chemkin form plus random thermochemical states,
all drawn from ``numpy.random.Generator(PCG64(seed))``.

This module holds no kinetics arithmetic.  It only draws numbers with the
shapes and value ranges of the paper's workloads; the CPU oracle and the HIP
path both consume its arrays.

Mechanism arrays (host, numpy):

=============  ==============  ================================================
name           shape / dtype   meaning
=============  ==============  ================================================
W              [K] f64         molar masses, g/mol
nasa7          [K,15] f64      Tmid, low-range a1..a7, high-range a1..a7
elem           [K,E] i32       element counts per species
rtype          [R] i32         0 elementary, 1 third-body, 2 Troe falloff
reac, prod     [R,3] i32       species index per molecule slot, -1 = empty
lnA, b, theta  [R] f64         k = exp(lnA) T^b exp(-theta/T), mol-cm-s units
eff            [R,K] f64       third-body efficiencies (1 if unused)
troe           [R,4] f64       alpha, T***, T*, T** (Troe only)
low            [R,3] f64       lnA0, b0, theta0 of the low-pressure limit
=============  ==============  ================================================
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

ATOMIC_WEIGHTS = np.array([12.011, 1.008, 15.999, 14.007])  # C, H, O, N
N_ELEMENTS = 4
MAX_ATOMS = 6
# temperature nodes of the heat-capacity draw (K)
_CP_NODES = np.array([300.0, 1000.0, 2000.0, 3500.0, 5000.0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _draw_species(rng, n_species, max_atoms=None):
    """Distinct element-count vectors with 1..max_atoms atoms (MAX_ATOMS by default).

    The single atoms come first; later species are preferentially sums of two
    existing species so that recombination and exchange reactions exist.
    """
    max_atoms = MAX_ATOMS if max_atoms is None else int(max_atoms)
    # small mechanisms use fewer elements (like H2/O2 chemistry), which gives
    # them enough element-balanced exchange reactions
    n_el = 2 if n_species <= 12 else (3 if n_species <= 30 else N_ELEMENTS)
    # distinct vectors with 1..max_atoms atoms over n_el elements
    n_distinct = math.comb(max_atoms + n_el, n_el) - 1
    if n_species > n_distinct:
        raise ValueError(f"{n_species} species need more than {max_atoms} atoms per species")
    comps = [tuple(int(i == e) for i in range(N_ELEMENTS)) for e in range(n_el)]
    seen = set(comps)
    while len(comps) < n_species:
        if rng.random() < 0.75 and len(comps) >= 2:
            i, j = rng.integers(0, len(comps), size=2)
            c = tuple(a + b for a, b in zip(comps[i], comps[j]))
        else:
            n_at = int(rng.integers(2, max_atoms + 1))
            c = tuple(np.bincount(rng.integers(0, n_el, size=n_at),
                                  minlength=N_ELEMENTS).tolist())
        if sum(c) > max_atoms or c in seen:
            continue
        seen.add(c)
        comps.append(c)
    return np.array(comps, dtype=np.int32)


def _draw_cp_nodes(rng, n_atoms):
    """Increasing cp/R values at the temperature nodes, in [2.5, 2.5 + 1.5 n]."""
    hi = 2.5 + 1.5 * n_atoms
    while True:
        v = np.sort(rng.uniform(2.5, hi, size=5))
        # quartic through the nodes, fitted in tau = T/1000 then rescaled
        tau = _CP_NODES / 1000.0
        V = np.vander(tau, 5, increasing=True)
        c = np.linalg.solve(V, v)
        a = c / (1000.0 ** np.arange(5))
        # reject draws whose quartic leaves (0.5, 2 hi) on [200, 6000] K
        tt = np.linspace(200.0, 6000.0, 233) / 1000.0
        vals = np.vander(tt, 5, increasing=True) @ c
        if vals.min() > 0.5 and vals.max() < 2.0 * hi:
            return a


def _pair_sums(comps):
    out = {}
    n = len(comps)
    for i in range(n):
        for j in range(i, n):
            out.setdefault(tuple((comps[i] + comps[j]).tolist()), []).append((i, j))
    return out


def make_mechanism(n_species: int, n_reactions: int, n_thirdbody: int, n_troe: int,
                   seed: int, hf_scale: float = 1.0, max_atoms: int | None = None) -> dict:
    """Draw an element-balanced, reversible mechanism.

    Elementary reactions are A+B<=>C+D with equal element totals on both sides;
    third-body and Troe reactions are A+B(+M)<=>AB(+M).  Every reaction is
    written in the direction in which the drawn formation enthalpies decrease,
    the way mechanisms usually list exothermic steps forward.  Arrhenius draws follow the configuration text:
    log10 A ~ U(8,14), b ~ U(-1,2), theta ~ U(0,25000) K.
    """
    rng = _rng(seed)
    comps = _draw_species(rng, n_species, max_atoms)
    K = n_species
    n_atoms = comps.sum(axis=1)
    W = comps @ ATOMIC_WEIGHTS

    nasa = np.zeros((K, 15))
    hf = np.zeros(K)
    T0 = 298.15
    for k in range(K):
        a = _draw_cp_nodes(rng, int(n_atoms[k]))
        # formation enthalpy h_f(298)/R ~ U(-1e5, 1e5) J/mol / R, and a standard
        # entropy that grows with molar mass and atom count the way tabulated
        # species data do (translational part ~ 1.5 ln W), plus noise
        hf[k] = hf_scale * rng.uniform(-1.0e5, 1.0e5) / 8.314462618
        s_target = 13.0 + 1.5 * np.log(W[k]) + 1.2 * (n_atoms[k] - 1) + rng.uniform(-1.0, 1.0)
        # a6, a7 place h/R and s/R of the drawn cp polynomial at those targets
        a6 = hf[k] - (a[0] * T0 + a[1] * T0**2 / 2 + a[2] * T0**3 / 3 + a[3] * T0**4 / 4
                      + a[4] * T0**5 / 5)
        a7 = s_target - (a[0] * np.log(T0) + a[1] * T0 + a[2] * T0**2 / 2 + a[3] * T0**3 / 3
                         + a[4] * T0**4 / 4)
        row = np.concatenate([a, [a6, a7]])
        nasa[k, 0] = 1000.0
        nasa[k, 1:8] = row
        nasa[k, 8:15] = row

    sums = _pair_sums(comps)
    comp_index = {tuple(c.tolist()): k for k, c in enumerate(comps)}
    exch = []   # ((i,j),(k,l))
    for key, pairs in sums.items():
        for x in range(len(pairs)):
            for y in range(x + 1, len(pairs)):
                exch.append((pairs[x], pairs[y]))
    recomb = []  # ((i,j), k) with comp(i)+comp(j) = comp(k)
    for key, pairs in sums.items():
        if key in comp_index:
            for p in pairs:
                recomb.append((p, comp_index[key]))
    n_el = n_reactions - n_thirdbody - n_troe
    if len(exch) < n_el or len(recomb) < n_thirdbody + n_troe:
        raise ValueError(f"seed {seed}: only {len(exch)} exchange / {len(recomb)} "
                         f"recombination candidates for {n_el} / {n_thirdbody + n_troe}")
    pick_e = rng.choice(len(exch), size=n_el, replace=False)
    pick_r = rng.choice(len(recomb), size=n_thirdbody + n_troe, replace=False)

    R = n_reactions
    rtype = np.zeros(R, np.int32)
    reac = -np.ones((R, 3), np.int32)
    prod = -np.ones((R, 3), np.int32)
    a6 = hf
    order = rng.permutation(R)  # interleave the reaction types like a real file
    slots = iter(order)
    for idx in pick_e:
        (i, j), (k, l) = exch[idx]
        r = next(slots)
        lhs, rhs = [i, j], [k, l]
        if a6[rhs].sum() > a6[lhs].sum():
            lhs, rhs = rhs, lhs
        reac[r, :2], prod[r, :2] = lhs, rhs
    for n_, idx in enumerate(pick_r):
        (i, j), k = recomb[idx]
        r = next(slots)
        rtype[r] = 1 if n_ < n_thirdbody else 2
        lhs, rhs = [i, j], [k]
        if a6[k] > a6[[i, j]].sum():
            lhs, rhs = rhs, lhs
        reac[r, :len(lhs)], prod[r, :len(rhs)] = lhs, rhs

    lnA = np.log(10.0) * rng.uniform(8.0, 14.0, size=R)
    b = rng.uniform(-1.0, 2.0, size=R)
    theta = rng.uniform(0.0, 25000.0, size=R)

    eff = np.ones((R, K))
    troe = np.zeros((R, 4))
    low = np.zeros((R, 3))
    for r in range(R):
        if rtype[r] == 0:
            continue
        sp = rng.choice(K, size=min(3, K), replace=False)
        eff[r, sp] = rng.uniform(0.5, 5.0, size=len(sp))
        if rtype[r] == 2:
            troe[r] = [rng.uniform(0.1, 0.9), rng.uniform(30.0, 300.0),
                       rng.uniform(500.0, 6000.0), rng.uniform(1000.0, 10000.0)]
            low[r] = [lnA[r] + np.log(10.0) * rng.uniform(3.0, 6.0),
                      rng.uniform(-2.0, 0.0), rng.uniform(0.0, theta[r])]
    return dict(n_species=K, n_reactions=R, n_elements=N_ELEMENTS, W=W,
                nasa7=nasa, elem=comps, rtype=rtype, reac=reac, prod=prod,
                lnA=lnA, b=b, theta=theta, eff=eff, troe=troe, low=low)


def make_states(mech: dict, n_cells: int, seed: int, T_ranges, fractions=None,
                alpha: float = 1.0, majors: int | None = None, floor: float = 0.0):
    """Cell states as a [N, n_cells] float64 SoA array (row 0 = T, rows 1.. = Y).

    ``T_ranges`` is a list of (lo, hi) uniform ranges mixed with ``fractions``.
    Y is Dirichlet(alpha) over all species, or over ``majors`` seeded species
    with ``floor`` on the others (then renormalised).
    """
    rng = _rng(seed)
    K = mech["n_species"]
    if fractions is None:
        fractions = [1.0 / len(T_ranges)] * len(T_ranges)
    counts = np.floor(np.asarray(fractions) * n_cells).astype(int)
    counts[-1] = n_cells - counts[:-1].sum()
    T = np.concatenate([rng.uniform(lo, hi, size=c) for (lo, hi), c in zip(T_ranges, counts)])
    T = T[rng.permutation(n_cells)]
    if majors is None:
        Y = rng.dirichlet(np.full(K, alpha), size=n_cells)
    else:
        sel = rng.choice(K, size=majors, replace=False)
        Y = np.full((n_cells, K), floor)
        Y[:, sel] = rng.dirichlet(np.full(majors, alpha), size=n_cells)
        Y /= Y.sum(axis=1, keepdims=True)
    out = np.empty((K + 1, n_cells))
    out[0] = T
    out[1:] = Y.T
    return out


@dataclass(frozen=True)
class Workload:
    """One benchmark configuration (sizes from the configuration list)."""
    name: str
    n_species: int
    n_reactions: int
    n_thirdbody: int
    n_troe: int
    n_cells: int
    p_pa: float
    dt: float
    T_ranges: tuple
    fractions: tuple | None
    mech_seed: int
    state_seed: int
    rtol: float = 1e-6
    atol: float = 1e-10
    alpha: float = 1.0
    majors: int | None = None
    floor: float = 0.0
    notes: str = ""
    pool: str | None = None  # file of pre-relaxed states to sample cells from
    ambient: str | None = None  # file of an ambient-zone state (zonal workload)
    ambient_frac: float = 0.0   # share of cells that are ambient
    ambient_jitter: float = 0.0  # ambient T = T_ambient + U(-jitter, jitter) K

    @property
    def N(self):
        return self.n_species + 1

    def mechanism(self) -> dict:
        return make_mechanism(self.n_species, self.n_reactions, self.n_thirdbody,
                              self.n_troe, self.mech_seed)

    def states(self, mech: dict | None = None, n_cells: int | None = None) -> np.ndarray:
        mech = mech if mech is not None else self.mechanism()
        if self.pool is not None:
            return pool_states(self.pool, n_cells or self.n_cells, self.state_seed)
        st = make_states(mech, n_cells or self.n_cells, self.state_seed, list(self.T_ranges),
                         self.fractions, self.alpha, self.majors, self.floor)
        if self.ambient is not None:
            # a seeded share of the cells is replaced by the ambient state with a
            # jittered temperature, scattered over the index range
            amb = np.load(os.path.join(POOL_DIR, self.ambient), allow_pickle=False)
            n = st.shape[1]
            rng = _rng(self.state_seed + 1)
            is_amb = rng.random(n) < self.ambient_frac
            jit = rng.uniform(-self.ambient_jitter, self.ambient_jitter, n)
            st[:, is_amb] = amb[:, None]
            st[0, is_amb] += jit[is_amb]
        return st

    def refmap_params(self) -> dict:
        """Reference-mapping parameters of a zonal workload: the indicator is the
        mass fraction of the species scarcest in the ambient state (absent from
        the zone, present in every reacting cell), the zone threshold is atol,
        and the temperature window is the ambient jitter."""
        amb = np.load(os.path.join(POOL_DIR, self.ambient), allow_pickle=False)
        w = np.zeros(self.n_species)
        w[int(np.argmin(amb[1:]))] = 1.0
        return dict(weight=w, z0=0.0, z_max=self.atol, dT=self.ambient_jitter)


POOL_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def pool_states(name: str, n_cells: int, seed: int) -> np.ndarray:
    """n_cells states drawn with replacement from a stored pool [N, P] (a .npy
    file next to the script that wrote it; see that script for its recipe)."""
    pool = np.load(os.path.join(POOL_DIR, name), allow_pickle=False)
    idx = _rng(seed).integers(0, pool.shape[1], size=n_cells)
    return np.ascontiguousarray(pool[:, idx])


ATM = 101325.0
WORKLOADS = {
    # 10 species / 27 reversible reactions, 4 of them third-body
    "c1_10sp": Workload("c1_10sp", 10, 27, 4, 0, 1024, ATM, 1e-6, ((900.0, 2500.0),), None,
                        1001, 2001),
    # 54 species / 270 reactions (27 third-body, 14 Troe), 60 bar, stratified states
    "c2_54sp": Workload("c2_54sp", 54, 270, 27, 14, 65536, 60e5, 1e-6,
                        ((700.0, 1000.0), (1800.0, 2600.0)), (0.8, 0.2), 1002, 2002),
    # batching workload: same mechanism, 262,144 cells, dt 1e-5 s, drawn from a
    # pool of states relaxed for different times (75% near equilibrium, 25%
    # mid-transient), so step counts span about 1 to 500
    "c3_batch": Workload("c3_batch", 54, 270, 27, 14, 262144, 60e5, 1e-5,
                         ((700.0, 1600.0),), None, 1002, 2003, pool="c3_relaxed_pool.npy"),
    # adjoint workload: 53 species / 325 reactions, 16,384 cells, 1 atm
    "c4_adj": Workload("c4_adj", 53, 325, 32, 16, 16384, ATM, 1e-6, ((1200.0, 2200.0),), None,
                       1004, 2004),
    # reference-mapping workload: the 54-species mechanism, 65,536 cells, 75% of
    # them an ambient zone (one near-equilibrium state, T jittered by +-2 K)
    # scattered among reacting cells drawn as in c2_54sp
    "zonal_54sp": Workload("zonal_54sp", 54, 270, 27, 14, 65536, 60e5, 1e-6,
                           ((700.0, 1000.0), (1800.0, 2600.0)), (0.8, 0.2), 1002, 2007,
                           ambient="zonal_ambient_state.npy", ambient_frac=0.75, ambient_jitter=2.0),
    # large mechanism: 150 species / 1000 reactions, 131,072 cells, 40 bar
    "c5_150sp": Workload("c5_150sp", 150, 1000, 100, 50, 131072, 40e5, 1e-6,
                         ((800.0, 2400.0),), None, 1005, 2005, alpha=0.5, majors=20,
                         floor=1e-12),
}


def objective_weights(n_species: int, seed: int = 4004) -> np.ndarray:
    """Weights w_k ~ U(0,1) of the adjoint objective sum_cells [T + sum_k w_k Y_k]."""
    return _rng(seed).uniform(0.0, 1.0, size=n_species)


def sha256_arrays(d: dict) -> str:
    h = hashlib.sha256()
    for k in sorted(d):
        v = d[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode())
            h.update(np.ascontiguousarray(v).tobytes())
    return h.hexdigest()
