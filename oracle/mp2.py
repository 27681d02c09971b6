"""Deterministic second-order energies for tiny inputs (Sec. II).

Test infrastructure: part of the FP64 oracle.

* ``spinor_eri``: Eq. transformation -- (pq|rs) = sum over the 16 component
  combinations (c, c' in {L alpha, L beta, S alpha, S beta}) of
  C^{c*}_{mu p} C^c_{nu q} C^{c'*}_{kappa r} C^{c'}_{lambda s} (mu nu|kappa lambda),
  with C^{L s} = C[s][L set], C^{S s} = C[s][S set] (coefficient block per spin).
* ``mp2_final``: Eq. FinalMP2 by explicit loops over i, j, a, b.
* ``mp2_spin_orbital``: the antisymmetrised textbook form
  (1/4) sum |<ij||ab>|^2 / (eps_i + eps_j - eps_a - eps_b), <ij|ab> = (ia|jb).
* ``mp2_closed_shell``: the nonrelativistic closed-shell textbook formula
  sum (ia|jb)[2(ia|jb) - (ib|ja)] / D over spatial orbitals.
"""
from __future__ import annotations

import numpy as np

from .eri import eri_full


def ao_eri(inp) -> np.ndarray:
    """(mu nu|kappa lambda) over the primitives, L-L and S-S distributions only."""
    nL, nb = inp.n_L, inp.n_b
    return eri_full(inp.prim_xyz, inp.prim_exp, inp.prim_lxyz, inp.prim_norm,
                    blocks=[range(0, nL), range(nL, nb)])


def spinor_eri(inp, ao: np.ndarray) -> np.ndarray:
    """(pq|rs) over all spinors [n_sp]^4."""
    nL, nb = inp.n_L, inp.n_b
    comps = []
    for s in range(2):
        for rng in (slice(0, nL), slice(nL, nb)):
            Cc = np.zeros((nb, inp.n_sp), dtype=complex)
            Cc[rng] = inp.coeffs[s, rng]
            comps.append(Cc)
    # B[mu, nu, p, q] = sum_c conj(C^c_{mu p}) C^c_{nu q}
    B = sum(np.einsum("mp,nq->mnpq", Cc.conj(), Cc) for Cc in comps)
    n2, s2 = nb * nb, inp.n_sp * inp.n_sp
    Bm = B.reshape(n2, s2)
    out = Bm.T @ ao.reshape(n2, n2) @ Bm
    return out.reshape(inp.n_sp, inp.n_sp, inp.n_sp, inp.n_sp)


def mp2_final_parts(eri: np.ndarray, eps: np.ndarray, n_occ: int):
    """Eq. FinalMP2 split into its direct and exchange sums:
    (1/2) sum (ia|jb)(ai|bj)/D and -(1/2) sum (ia|jb)(bi|aj)/D."""
    n = eps.shape[0]
    direct = 0.0 + 0.0j
    exchange = 0.0 + 0.0j
    for i in range(n_occ):
        for j in range(n_occ):
            for a in range(n_occ, n):
                for b in range(n_occ, n):
                    den = eps[i] + eps[j] - eps[a] - eps[b]
                    direct += eri[i, a, j, b] * eri[a, i, b, j] / den
                    exchange -= eri[i, a, j, b] * eri[b, i, a, j] / den
    return 0.5 * direct, 0.5 * exchange


def mp2_final(eri: np.ndarray, eps: np.ndarray, n_occ: int) -> complex:
    """Eq. FinalMP2."""
    d, x = mp2_final_parts(eri, eps, n_occ)
    return d + x


def mp2_spin_orbital(eri: np.ndarray, eps: np.ndarray, n_occ: int) -> float:
    """(1/4) sum_{ijab} |<ij||ab>|^2 / D with <ij|ab> = (ia|jb)."""
    o = slice(0, n_occ)
    v = slice(n_occ, eps.shape[0])
    g = eri[o, v, o, v].transpose(0, 2, 1, 3)          # <ij|ab> = (ia|jb)
    anti = g - g.transpose(0, 1, 3, 2)                  # <ij|ab> - <ij|ba>
    eo, ev = eps[o], eps[v]
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return float(0.25 * np.sum(np.abs(anti) ** 2 / D))


def mp2_closed_shell(inp, ao: np.ndarray) -> float:
    """Nonrelativistic closed-shell MP2 for inputs built in the 'nr' mode
    (spinor 2k = alpha psi_k, 2k+1 = beta psi_k, psi_k real on the L set)."""
    nL = inp.n_L
    psi = inp.coeffs[0, :nL, 0::2].real                  # [n_L, n_sp/2]
    e = inp.eps[0::2]
    no = inp.n_occ // 2
    aoL = ao[:nL, :nL, :nL, :nL]
    mo = np.einsum("mp,nq,kr,ls,mnkl->pqrs", psi, psi, psi, psi, aoL, optimize=True)
    total = 0.0
    nsp = e.shape[0]
    for i in range(no):
        for j in range(no):
            for a in range(no, nsp):
                for b in range(no, nsp):
                    total += mo[i, a, j, b] * (2.0 * mo[i, a, j, b] - mo[i, b, j, a]) / (e[i] + e[j] - e[a] - e[b])
    return total
