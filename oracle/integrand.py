"""The MC-MP2 integrand and the per-step redundant-walker estimator (Sec. III).

Test infrastructure: part of the FP64 oracle.  Written in plain PyTorch CPU
ops (complex128) so that reverse-mode differentiation of the very same code
gives the oracle's gradients.

Definitions followed
--------------------
Spinor values, Eq. (C):  phi_k^{L s}(r) = sum_{mu in L} C[s][mu][k] chi_mu(r),
phi_k^{S s}(r) = sum_{mu in S} C[s][mu][k] chi_mu(r), components ordered
(L alpha, L beta, S alpha, S beta).  The paper prints one coefficient C^L for
both spins; the reading adopted is a coefficient block per spin.

Green's functions (Sec. III):
    G-(x, y)_{cc'} = sum_i phi_i^c(x) conj(phi_i^{c'}(y)) exp(+eps_i tau)   [= G-(x, y, -tau)]
    G+(x, y)_{cc'} = sum_a phi_a^c(x) conj(phi_a^{c'}(y)) exp(-eps_a tau)

Integrand.  Inserting the Laplace transform of 1/(eps_i+eps_j-eps_a-eps_b)
into Eq. FinalMP2 and grouping the orbital sums of the products of
rho_pq(r) = phi_p^dagger(r) phi_q(r) gives, for points 1, 2, 3, 4,
    direct:   D = Tr[G-(3,1) G+(1,3)] * Tr[G-(4,2) G+(2,4)]
    exchange: X = Tr[G-(3,1) G+(1,4) G-(4,2) G+(2,3)]
    f = -(1/2) (D - X) / (r12 r34).
The printed Eq. MCMP2 writes these factors as vec(.)^T vec(.) dot products
with prefactors -2 and +1; for 4x4 spinor blocks summed over all spinors the
contraction that reproduces Eq. FinalMP2 is the trace form above (the
printed form is kept only as ``printed_form`` for a negative control).

Interaction (Sec. II): g(1, 2) = 1/r12 - alpha(1).alpha(2) / (2 r12)
- (alpha(1).r12)(alpha(2).r12) / (2 r12^3); the paper keeps only the first
(Coulomb) term.  Written as g = sum_{mu nu} W_{mu nu}(r12) s_mu(1) s_nu(2)
with s_0 = 1 (4x4) and s_k = alpha_k (Eq. alpha): W_00 = 1/r,
W_kl = -(delta_kl / r + c r_k r_l / r^3) / 2 (c = 1 with the second Breit
term, "breit"; c = 0 for the Gaunt term alone, "gaunt"), W_0k = W_k0 = 0.
Inserting s_mu into the orbital-density products rho_pq = phi_p^dagger s_mu phi_q
of the same grouping gives, with s_rho, s_sig acting at points 3, 4,
    D = sum W12[mu nu] W34[rho sig] Tr[G-(3,1) s_mu G+(1,3) s_rho] Tr[G-(4,2) s_nu G+(2,4) s_sig]
    X = sum W12[mu nu] W34[rho sig] Tr[G-(3,1) s_mu G+(1,4) s_sig G-(4,2) s_nu G+(2,3) s_rho]
    f = -(1/2) (D - X),
which for the Coulomb term alone is the form above.

Estimator, Eq. redundant: with m walker pairs (r1p, r2p),
    I'_n = (1/mC2) sum_{p<q} f(r1p, r2p, r1q, r2q, tau) / (w(r1p, r2p) w(r1q, r2q) w(tau)),
real part taken (the imaginary part of each term changes sign under p <-> q).
Several tau per step are averaged.
"""
from __future__ import annotations

import numpy as np
import torch

from .basis import basis_values
from .weights import g_values, pair_weight, tau_weight

CDT = torch.complex128
RDT = torch.float64


def spinor_values(points: np.ndarray, inp, coeffs: torch.Tensor = None) -> torch.Tensor:
    """phi[P, 4, n_sp] at points [P, 3] (Eq. (C))."""
    X = torch.from_numpy(basis_values(points, inp.prim_xyz, inp.prim_exp, inp.prim_lxyz, inp.prim_norm))
    C = torch.as_tensor(inp.coeffs) if coeffs is None else coeffs
    nL = inp.n_L
    XL = X[:, :nL].to(CDT)
    XS = X[:, nL:].to(CDT)
    return torch.stack([XL @ C[0, :nL], XL @ C[1, :nL], XS @ C[0, nL:], XS @ C[1, nL:]], dim=1)


def green_matrix(phi: torch.Tensor, e: torch.Tensor) -> torch.Tensor:
    """G[x, c, y, c'] = sum_k phi[x, c, k] e[k] conj(phi[y, c', k])."""
    P, nc, n = phi.shape
    A = phi.reshape(P * nc, n)
    G = (A * e.to(CDT)) @ A.conj().transpose(0, 1)
    return G.reshape(P, nc, P, nc)


def _blk(G: torch.Tensor, x, y) -> torch.Tensor:
    """4x4 blocks G(x, y) for index arrays x, y -> [Q, 4, 4]."""
    return G[x, :, y, :]


def _tr(A: torch.Tensor) -> torch.Tensor:
    return torch.diagonal(A, dim1=-2, dim2=-1).sum(-1)


def direct_exchange(Gm: torch.Tensor, Gp: torch.Tensor, i1, i2, i3, i4):
    """(D, X) of the trace-form integrand for point quadruples (i1, i2, i3, i4)."""
    D = _tr(_blk(Gm, i3, i1) @ _blk(Gp, i1, i3)) * _tr(_blk(Gm, i4, i2) @ _blk(Gp, i2, i4))
    X = _tr(_blk(Gm, i3, i1) @ _blk(Gp, i1, i4) @ _blk(Gm, i4, i2) @ _blk(Gp, i2, i3))
    return D, X


def dirac_matrices() -> torch.Tensor:
    """s[mu] for mu = 0..3: the 4x4 identity and alpha_k = [[0, sigma_k], [sigma_k, 0]]
    (Eq. alpha), components (L alpha, L beta, S alpha, S beta)."""
    pauli = [np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
             np.array([[1, 0], [0, -1]], dtype=complex)]
    s = np.zeros((4, 4, 4), dtype=complex)
    s[0] = np.eye(4)
    for k in range(3):
        s[k + 1, :2, 2:] = pauli[k]
        s[k + 1, 2:, :2] = pauli[k]
    return torch.from_numpy(s)


INTERACTIONS = ("coulomb", "gaunt", "breit")


def interaction_weights(r12: torch.Tensor, kind: str) -> torch.Tensor:
    """W[Q, 4, 4] (real) of g = sum W_{mu nu}(r12) s_mu(1) s_nu(2) for vectors r12 [Q, 3]."""
    if kind not in INTERACTIONS:
        raise ValueError(kind)
    r = torch.linalg.norm(r12, dim=-1)
    W = torch.zeros(r12.shape[0], 4, 4, dtype=RDT)
    W[:, 0, 0] = 1.0 / r
    if kind != "coulomb":
        eye = torch.eye(3, dtype=RDT)
        W[:, 1:, 1:] = -0.5 * eye / r[:, None, None]
        if kind == "breit":
            W[:, 1:, 1:] -= 0.5 * r12[:, :, None] * r12[:, None, :] / (r ** 3)[:, None, None]
    return W


def direct_exchange_general(Gm: torch.Tensor, Gp: torch.Tensor, i1, i2, i3, i4, W12: torch.Tensor,
                            W34: torch.Tensor):
    """(D, X) for the interaction sum W_{mu nu} s_mu s_nu on the pairs (1, 2)
    and (3, 4), weights included (W12, W34: [Q, 4, 4])."""
    s = dirac_matrices()
    A31, P13 = _blk(Gm, i3, i1), _blk(Gp, i1, i3)
    A42, P24 = _blk(Gm, i4, i2), _blk(Gp, i2, i4)
    P14, P23 = _blk(Gp, i1, i4), _blk(Gp, i2, i3)
    Wc12, Wc34 = W12.to(CDT), W34.to(CDT)
    # T1[mu, rho] = Tr[G-(3,1) s_mu G+(1,3) s_rho], T2[nu, sig] = Tr[G-(4,2) s_nu G+(2,4) s_sig]
    T1 = torch.einsum("qab,mbc,qcd,rda->qmr", A31, s, P13, s)
    T2 = torch.einsum("qab,nbc,qcd,sda->qns", A42, s, P24, s)
    D = torch.einsum("qmn,qrs,qmr,qns->q", Wc12, Wc34, T1, T2)
    # L[mu, sig] = G-(3,1) s_mu G+(1,4) s_sig, R[nu, rho] = G-(4,2) s_nu G+(2,3) s_rho
    L = torch.einsum("qab,mbc,qcd,sde->qmsae", A31, s, P14, s)
    R = torch.einsum("qab,nbc,qcd,rde->qnrae", A42, s, P23, s)
    X = torch.einsum("qmn,qrs,qmsab,qnrba->q", Wc12, Wc34, L, R)
    return D, X


def printed_form(Gm: torch.Tensor, Gp: torch.Tensor, i1, i2, i3, i4):
    """Eq. MCMP2 read literally (vec^T vec products, prefactors -2 and +1),
    without the 1/(r12 r34) factor.  Kept only as a negative control."""
    def vdot(A, B):
        return (A * B).sum(dim=(-2, -1))
    t1 = vdot(_blk(Gm, i1, i3), _blk(Gp, i3, i1)) * vdot(_blk(Gm, i2, i4), _blk(Gp, i4, i2))
    t2 = vdot(_blk(Gm, i1, i3), _blk(Gp, i4, i1)) * vdot(_blk(Gm, i2, i4), _blk(Gp, i3, i2))
    return -2.0 * t1 + t2


def tau_factors(eps: torch.Tensor, n_occ: int, tau: float):
    """exp(+eps_i tau) for occupied, exp(-eps_a tau) for virtual spinors."""
    return torch.exp(eps[:n_occ] * tau), torch.exp(-eps[n_occ:] * tau)


def step_estimate(inp, walkers: np.ndarray, taus, lam: float, Ng: float,
                  coeffs: torch.Tensor = None, eps: torch.Tensor = None, return_pairs: bool = False,
                  interaction: str = "coulomb"):
    """Per-step estimate of Eq. redundant at fixed walkers and tau samples,
    with the Coulomb interaction (the paper's) or Coulomb plus the Gaunt term
    or plus both Breit terms of the interaction operator of Sec. II.

    Returns a real tensor [n_tau, 3] whose columns are the direct part
    Re(-D/2 ...), the exchange part Re(+X/2 ...) and their sum, each already
    divided by the weights and averaged over the mC2 walker pairs.
    With return_pairs=True also returns the complex per-pair quotients
    f / (w_p w_q w_tau) as a list over tau.
    """
    walkers = np.asarray(walkers, dtype=float)
    m = walkers.shape[0]
    pts = walkers.reshape(2 * m, 3)
    C = torch.as_tensor(inp.coeffs) if coeffs is None else coeffs
    e = torch.as_tensor(inp.eps) if eps is None else eps
    phi = spinor_values(pts, inp, C)
    no = inp.n_occ
    P, Q = torch.triu_indices(m, m, offset=1)
    i1, i2, i3, i4 = 2 * P, 2 * P + 1, 2 * Q, 2 * Q + 1
    r12v = torch.from_numpy(walkers[:, 0] - walkers[:, 1])
    r12 = torch.linalg.norm(r12v, dim=-1)
    if interaction != "coulomb":
        W = interaction_weights(r12v, interaction)
    w = torch.from_numpy(pair_weight(walkers[:, 0], walkers[:, 1], inp.nuc_xyz, inp.wfn, Ng))
    out = []
    pairs = []
    for tau in np.atleast_1d(np.asarray(taus, dtype=float)):
        eo, ev = tau_factors(e, no, float(tau))
        Gm = green_matrix(phi[:, :, :no], eo)
        Gp = green_matrix(phi[:, :, no:], ev)
        wt = float(tau_weight(tau, lam))
        if interaction == "coulomb":
            D, X = direct_exchange(Gm, Gp, i1, i2, i3, i4)
            scale = 1.0 / (r12[P] * r12[Q]) / (w[P] * w[Q] * wt)
        else:
            D, X = direct_exchange_general(Gm, Gp, i1, i2, i3, i4, W[P], W[Q])
            scale = 1.0 / (w[P] * w[Q] * wt)
        q_dir = -0.5 * D * scale
        q_exc = 0.5 * X * scale
        d = q_dir.real.mean()
        x = q_exc.real.mean()
        out.append(torch.stack([d, x, d + x]))
        if return_pairs:
            pairs.append(q_dir + q_exc)
    res = torch.stack(out)
    return (res, pairs) if return_pairs else res


def walker_g(walkers: np.ndarray, inp) -> np.ndarray:
    """g(r1p) g(r2p) per pair (used by tests of the 1/r cancellation)."""
    return g_values(walkers[:, 0], inp.nuc_xyz, inp.wfn) * g_values(walkers[:, 1], inp.nuc_xyz, inp.wfn)
