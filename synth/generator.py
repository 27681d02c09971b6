"""Synthetic heavy-molecule-shaped inputs (stand-ins for the paper's DHF data).

The paper's own inputs (UTChem basis files and DHF spinor coefficients for
H2 ... Au2, Sec. IV) are not available, so every workload here is fabricated
from a fixed seed with the shapes the method sees:

* nuclei on a compact cluster with the Au2 bond length of Sec. IV (2.59 A =
  4.894 bohr) as edge;
* a Cartesian primitive large-component (L) set of s/p/d shells with
  log-uniform exponents, and the small-component (S) set that kinetic balance
  (Sec. II, i(sigma.p) acting on the L functions) requires: every L shell of
  angular momentum l on centre A with exponent z contributes S shells
  (A, z, l+1) and, for l >= 1, (A, z, l-1) -- the unrestricted kinetic-balance
  span;
* spinor coefficients C[s][mu][k] (s = alpha, beta; mu over L then S) that
  come in Kramers pairs (partner of (c_a, c_b) is (-conj c_b, conj c_a)),
  with the S block scaled by kappa_S and the whole set Loewdin-orthonormalised
  in the four-component overlap metric blockdiag(S_LL, S_SS) per spin;
* spinor energies drawn per Kramers pair, occupied in [-3, -0.5] Eh and
  virtual in [0.2, 5] Eh, ascending within each group;
* the electron-pair weight-function parameters of Table 1 (the Ag row,
  c1 = 0.1, zeta1 = 0.1, c2 = 0.8, zeta2 = 0.6) on every nucleus.

Only input fabrication happens here (primitive normalisation and overlaps for
the orthonormalisation); nothing of the MC-MP2 estimator is computed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
AU2_EDGE = 2.59 * BOHR_PER_ANGSTROM  # 4.894 bohr
AG_WEIGHT_ROW = (0.1, 0.1, 0.8, 0.6)  # Table 1: c1, zeta1, c2, zeta2 for Ag

# Seed streams of numpy.random.SeedSequence([seed, stream]).
STREAM_SHELLS, STREAM_COEFFS, STREAM_EPS, STREAM_PROBES, STREAM_WALKERS = 0, 1, 2, 3, 4


def cartesian_components(l: int) -> List[Tuple[int, int, int]]:
    """Cartesian exponent triples of a shell of total angular momentum l,
    in the order xx..x first (lx descending, then ly descending)."""
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def _geometry(kind: str, n_nuc: int) -> np.ndarray:
    a = AU2_EDGE
    if kind == "pair":
        return np.array([[0.0, 0.0, -0.75], [0.0, 0.0, 0.75]])
    if kind == "triangle":
        rc = a / math.sqrt(3.0)
        return np.array([[rc * math.cos(2 * math.pi * i / 3), rc * math.sin(2 * math.pi * i / 3), 0.0]
                         for i in range(3)])
    if kind == "tetrahedron":
        s = a / math.sqrt(8.0)
        return s * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    if kind == "octahedron":
        s = a / math.sqrt(2.0)
        return s * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                            dtype=float)
    raise ValueError(kind)


# name -> workload description.  shells: list of (nucleus, l) in order.
CONFIGS: Dict[str, dict] = {
    # Tiny plain FP64: 2 nuclei 1.5 bohr apart, per nucleus 3 s + 1 p L shells.
    "C0": dict(geometry="pair", n_nuc=2, shell_plan=("per_nucleus", (0, 0, 0, 1)),
               exp_range=(0.1, 20.0), n_occ=4, n_vir=16, m=16, n_tau=1),
    # Plain FP64 GPU baseline: 3 nuclei, (s,p,d) x 20 shells -> 200 L primitives.
    "C1": dict(geometry="triangle", n_nuc=3, shell_plan=("cycle", (0, 1, 2), 20),
               exp_range=(0.05, 5000.0), n_occ=40, n_vir=300, m=128, n_tau=2),
    # Differentiation: C1 sizes with gradients.
    "C2": dict(geometry="triangle", n_nuc=3, shell_plan=("cycle", (0, 1, 2), 20),
               exp_range=(0.05, 5000.0), n_occ=40, n_vir=300, m=128, n_tau=2),
    # Precision: 4 nuclei, 600 L primitives.
    "C3": dict(geometry="tetrahedron", n_nuc=4, shell_plan=("cycle", (0, 1, 2), 60),
               exp_range=(0.05, 5000.0), n_occ=80, n_vir=900, m=256, n_tau=1),
    # Largest: 6 nuclei, 1000 L primitives.
    "C4": dict(geometry="octahedron", n_nuc=6, shell_plan=("cycle", (0, 1, 2), 100),
               exp_range=(0.05, 5000.0), n_occ=120, n_vir=1500, m=512, n_tau=4),
}


@dataclasses.dataclass
class Inputs:
    """Everything the MC-MP2 step consumes, in host memory (float64 / complex128).

    Attributes
    ----------
    nuc_xyz   : [n_nuc, 3] nuclear positions (bohr)
    wfn       : [n_nuc, 4] weight-function parameters (c1, zeta1, c2, zeta2), Eq. basisSet
    n_L, n_S  : numbers of Cartesian primitives in the large and small sets
    prim_xyz  : [n_b, 3] primitive centres, L set first, n_b = n_L + n_S
    prim_exp  : [n_b] exponents
    prim_lxyz : [n_b, 3] Cartesian powers (int32)
    prim_norm : [n_b] normalisation constants (each primitive has unit L2 norm)
    coeffs    : [2, n_b, n_sp] complex spinor coefficients C[spin][mu][k]
    eps       : [n_sp] spinor energies, occupied first, Kramers partners adjacent
    n_occ, n_vir, m, n_tau : sizes
    """
    name: str
    nuc_xyz: np.ndarray
    wfn: np.ndarray
    n_L: int
    n_S: int
    prim_xyz: np.ndarray
    prim_exp: np.ndarray
    prim_lxyz: np.ndarray
    prim_norm: np.ndarray
    coeffs: np.ndarray
    eps: np.ndarray
    n_occ: int
    n_vir: int
    m: int
    n_tau: int
    shell_of_prim: np.ndarray = None

    @property
    def n_b(self) -> int:
        return self.n_L + self.n_S

    @property
    def n_sp(self) -> int:
        return self.n_occ + self.n_vir

    def with_(self, **kw) -> "Inputs":
        return dataclasses.replace(self, **kw)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed, stream]))


def _double_factorial_odd(n: int) -> int:
    """(2n-1)!! for n >= 0, with (-1)!! = 1."""
    out = 1
    for k in range(1, 2 * n, 2):
        out *= k
    return out


def primitive_norm(alpha: np.ndarray, lxyz: np.ndarray) -> np.ndarray:
    """Unit-L2 normalisation of (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-alpha r^2)."""
    L = lxyz.sum(axis=1)
    df = np.array([_double_factorial_odd(int(a)) * _double_factorial_odd(int(b)) * _double_factorial_odd(int(c))
                   for a, b, c in lxyz], dtype=float)
    return np.sqrt((2.0 * alpha / np.pi) ** 1.5 * (4.0 * alpha) ** L / df)


def _overlap_1d_table(lmax: int, a, b, A, B) -> np.ndarray:
    """Obara-Saika 1D overlap table s[i][j] (i, j <= lmax) for unnormalised
    Cartesian Gaussians, vectorised over the leading axis of a, b, A, B."""
    p = a + b
    mu = a * b / p
    P = (a * A + b * B) / p
    XPA, XPB, XAB = P - A, P - B, A - B
    n = a.shape[0]
    s = np.zeros((lmax + 1, lmax + 1, n))
    s[0, 0] = np.sqrt(np.pi / p) * np.exp(-mu * XAB * XAB)
    inv2p = 0.5 / p
    for i in range(lmax + 1):
        for j in range(lmax + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = XPA * s[i - 1, j]
                if i > 1:
                    v = v + (i - 1) * inv2p * s[i - 2, j]
                if j > 0:
                    v = v + j * inv2p * s[i - 1, j - 1]
            else:
                v = XPB * s[i, j - 1]
                if j > 1:
                    v = v + (j - 1) * inv2p * s[i, j - 2]
            s[i, j] = v
    return s


def overlap_matrix(xyz: np.ndarray, alpha: np.ndarray, lxyz: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """Overlap of normalised Cartesian primitives (dense [n, n])."""
    n = alpha.shape[0]
    lmax = int(lxyz.max()) if n else 0
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    S = np.ones(ii.shape[0])
    for d in range(3):
        tab = _overlap_1d_table(lmax, alpha[ii], alpha[jj], xyz[ii, d], xyz[jj, d])
        S = S * tab[lxyz[ii, d], lxyz[jj, d], np.arange(ii.shape[0])]
    S = S * norm[ii] * norm[jj]
    return S.reshape(n, n)


def _build_basis(cfg: dict, seed: int):
    nuc = _geometry(cfg["geometry"], cfg["n_nuc"])
    plan = cfg["shell_plan"]
    if plan[0] == "per_nucleus":
        shells = [(I, l) for I in range(cfg["n_nuc"]) for l in plan[1]]
    else:  # ("cycle", ls, reps): rep r places one shell of every l on nucleus r % n_nuc
        _, ls, reps = plan
        shells = [(r % cfg["n_nuc"], l) for r in range(reps) for l in ls]
    lo, hi = cfg["exp_range"]
    rng = _rng(seed, STREAM_SHELLS)
    exps = np.exp(rng.uniform(math.log(lo), math.log(hi), size=len(shells)))
    L_shells = [(I, l, float(z)) for (I, l), z in zip(shells, exps)]
    S_shells = []
    seen = set()
    for I, l, z in L_shells:
        for ls in ((l + 1, l - 1) if l >= 1 else (l + 1,)):
            key = (I, ls, z)
            if key not in seen:
                seen.add(key)
                S_shells.append(key)
    prims = []  # (xyz, exp, lxyz, shell id)
    for sid, (I, l, z) in enumerate(L_shells + S_shells):
        for c in cartesian_components(l):
            prims.append((nuc[I], z, c, sid))
    n_L = sum(len(cartesian_components(l)) for _, l, _ in L_shells)
    xyz = np.array([p[0] for p in prims], dtype=float)
    alpha = np.array([p[1] for p in prims], dtype=float)
    lxyz = np.array([p[2] for p in prims], dtype=np.int32)
    shell = np.array([p[3] for p in prims], dtype=np.int32)
    return nuc, n_L, len(prims) - n_L, xyz, alpha, lxyz, shell


def _loewdin(C: np.ndarray, S_blocks: Tuple[np.ndarray, np.ndarray], n_L: int) -> np.ndarray:
    """C <- C (C^H S C)^(-1/2) with S = blockdiag(S_LL, S_SS) for each spin."""
    S_LL, S_SS = S_blocks
    M = np.zeros((C.shape[2], C.shape[2]), dtype=complex)
    for s in range(2):
        CL, CS = C[s, :n_L], C[s, n_L:]
        M += CL.conj().T @ (S_LL @ CL) + CS.conj().T @ (S_SS @ CS)
    M = 0.5 * (M + M.conj().T)
    w, U = np.linalg.eigh(M)
    if w.min() <= 1e-10 * w.max():
        raise RuntimeError("coefficient set is numerically linearly dependent")
    Minvh = (U * (1.0 / np.sqrt(w))) @ U.conj().T
    return C @ Minvh


def make_inputs(name: str = "C0", seed: int = 0, kappa_s: float = 0.1, mode: str = "dirac",
                n_occ: int = None, n_vir: int = None, m: int = None, n_tau: int = None,
                exp_range: Tuple[float, float] = None, shell_reps: int = None) -> Inputs:
    """Build the synthetic workload `name` (C0..C4).

    mode = "dirac": general complex four-component Kramers pairs (S block
    scaled by kappa_s before orthonormalisation).
    mode = "nr": nonrelativistic limit -- real spatial orbitals on the L set,
    spinors (psi, 0, 0, 0) and (0, psi, 0, 0); the S block is zero.
    mode = "2c": general complex Kramers pairs with a zero S block.
    """
    cfg = dict(CONFIGS[name])
    for k, v in (("n_occ", n_occ), ("n_vir", n_vir), ("m", m), ("n_tau", n_tau), ("exp_range", exp_range)):
        if v is not None:
            cfg[k] = v
    if shell_reps is not None:  # a "cycle" plan with another number of repetitions (basis-size ladders)
        kind, ls, _ = cfg["shell_plan"]
        if kind != "cycle":
            raise ValueError("shell_reps applies to workloads with a cycle shell plan")
        cfg["shell_plan"] = (kind, ls, int(shell_reps))
    if cfg["n_occ"] % 2 or cfg["n_vir"] % 2:
        raise ValueError("Kramers pairs need even n_occ and n_vir")
    nuc, n_L, n_S, xyz, alpha, lxyz, shell = _build_basis(cfg, seed)
    norm = primitive_norm(alpha, lxyz)
    n_b = n_L + n_S
    n_occ, n_vir = cfg["n_occ"], cfg["n_vir"]
    n_sp = n_occ + n_vir
    rng = _rng(seed, STREAM_COEFFS)
    S_LL = overlap_matrix(xyz[:n_L], alpha[:n_L], lxyz[:n_L], norm[:n_L])
    S_SS = overlap_matrix(xyz[n_L:], alpha[n_L:], lxyz[n_L:], norm[n_L:])
    if mode == "nr":
        psi = rng.standard_normal((n_L, n_sp // 2))
        w, U = np.linalg.eigh(psi.T @ S_LL @ psi)
        psi = psi @ ((U / np.sqrt(w)) @ U.T)
        C = np.zeros((2, n_b, n_sp), dtype=complex)
        C[0, :n_L, 0::2] = psi
        C[1, :n_L, 1::2] = psi
    else:
        half = n_sp // 2
        par = (rng.standard_normal((2, n_b, half)) + 1j * rng.standard_normal((2, n_b, half))) / math.sqrt(2.0)
        ks = 0.0 if mode == "2c" else kappa_s
        par[:, n_L:, :] *= ks
        C = np.zeros((2, n_b, n_sp), dtype=complex)
        C[:, :, 0::2] = par
        C[0, :, 1::2] = -np.conj(par[1])
        C[1, :, 1::2] = np.conj(par[0])
        C = _loewdin(C, (S_LL, S_SS), n_L)
    rng = _rng(seed, STREAM_EPS)
    eo = np.sort(rng.uniform(-3.0, -0.5, size=n_occ // 2))
    ev = np.sort(rng.uniform(0.2, 5.0, size=n_vir // 2))
    eps = np.concatenate([np.repeat(eo, 2), np.repeat(ev, 2)])
    wfn = np.tile(np.array(AG_WEIGHT_ROW, dtype=float), (cfg["n_nuc"], 1))
    return Inputs(name=name, nuc_xyz=nuc, wfn=wfn, n_L=n_L, n_S=n_S, prim_xyz=xyz, prim_exp=alpha,
                  prim_lxyz=lxyz, prim_norm=norm, coeffs=C, eps=eps, n_occ=n_occ, n_vir=n_vir,
                  m=cfg["m"], n_tau=cfg["n_tau"], shell_of_prim=shell)


def initial_walkers(inp: Inputs, seed: int = 0, chain: int = 0, m: int = None) -> np.ndarray:
    """Starting electron-pair positions [m, 2, 3]: each electron sits on a
    uniformly chosen nucleus plus a normal offset of variance 1/(2 zeta2)
    per coordinate (the tighter Gaussian of that nucleus's weight function)."""
    m = inp.m if m is None else m
    rng = np.random.default_rng(np.random.SeedSequence([seed, STREAM_WALKERS, chain]))
    I = rng.integers(0, inp.nuc_xyz.shape[0], size=(m, 2))
    sd = np.sqrt(1.0 / (2.0 * inp.wfn[I, 3]))
    return inp.nuc_xyz[I] + rng.standard_normal((m, 2, 3)) * sd[..., None]


def probe_rng(seed: int = 0) -> np.random.Generator:
    """Generator for finite-difference probe indices."""
    return _rng(seed, STREAM_PROBES)
