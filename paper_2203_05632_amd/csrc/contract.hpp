// Per-walker-pair contraction of the MC-MP2 integrand from G tiles in LDS
// (shared by the FP64 and the low-precision Green's-function kernels).  See
// green.hip for the definitions.
#pragma once

#include <type_traits>

#include "internal.hpp"

// complex numbers in the contraction's arithmetic type F (FP64, or FP32 in
// the BF16 / FP16 modes)
template <typename F>
struct cx {
    F re, im;
};
using cplx = cx<double>;
template <typename F>
__device__ inline cx<F> cmul(cx<F> a, cx<F> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename F>
__device__ inline cx<F> cmulc(cx<F> a, cx<F> b) {  // conj(a) * b
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename F>
__device__ inline cx<F> cadd(cx<F> a, cx<F> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename F>
__device__ inline cx<F> csub(cx<F> a, cx<F> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename F>
__device__ inline cx<F> conjc(cx<F> a) {
    return {a.re, -a.im};
}
template <typename F>
__device__ inline cx<F> shfl_xor_c(cx<F> a, int mask) {
    return {__shfl_xor(a.re, mask, 64), __shfl_xor(a.im, mask, 64)};
}

// Lane moves within 16-lane rows by DPP (a VALU operand modifier, no LDS
// traffic): CTRL 0x00-0xFF = quad_perm, 0x128 = row_ror:8, 0x141 =
// row_half_mirror.
template <int CTRL>
__device__ inline float dpp(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp(double x) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)v, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL, typename F>
__device__ inline cx<F> dpp_c(cx<F> a) {
    return {dpp<CTRL>(a.re), dpp<CTRL>(a.im)};
}
// Sum over the 16 lanes of each row, the same bits in every lane: xor 8
// (row_ror:8), then lane j <-> 7 - j within each half row (row_half_mirror),
// xor 1, xor 2 -- each step adds a value and its partner's, so the two
// lanes of a pair compute the same sum.
template <typename F>
__device__ inline cx<F> row16_sum(cx<F> v) {
    v = cadd(v, dpp_c<0x128>(v));
    v = cadd(v, dpp_c<0x141>(v));
    v = cadd(v, dpp_c<0xB1>(v));
    v = cadd(v, dpp_c<0x4E>(v));
    return v;
}
// Lane l of each group of four consecutive lanes, in all four (quad_perm [l, l, l, l]).
template <int L, typename F>
__device__ inline cx<F> quad_bcast(cx<F> a) {
    return dpp_c<0x55 * L>(a);
}
// The value of lane `l` (wave-uniform).
__device__ inline double lane_value(double x, int l) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <typename F>
__device__ inline cx<F> shfl_c(cx<F> a, int src) {
    return {__shfl(a.re, src, 64), __shfl(a.im, src, 64)};
}

// Adjoint-block element stores: FP64 complex, or a BF16 pair packed in 32
// bits (real part in the low half), rounded to nearest even.
__device__ inline void h_store(double2 *H, size_t i, double re, double im) { H[i] = double2{re, im}; }
__device__ inline uint32_t bf16_pair(float re, float im) {
    const __bf16 r = (__bf16)re, m = (__bf16)im;
    return (uint32_t)__builtin_bit_cast(unsigned short, r) | ((uint32_t)__builtin_bit_cast(unsigned short, m) << 16);
}
__device__ inline void h_store(uint32_t *H, size_t i, double re, double im) {
    const __bf16 r = (__bf16)(float)re, m = (__bf16)(float)im;
    H[i] = (uint32_t)__builtin_bit_cast(unsigned short, r) | ((uint32_t)__builtin_bit_cast(unsigned short, m) << 16);
}


template <typename F>
__device__ inline cx<F> to_cx(const cplx &v) {
    return {(F)v.re, (F)v.im};
}
template <typename F>
__device__ inline cx<F> to_cx(const float2 &v) {
    return {(F)v.x, (F)v.y};
}

// One walker pair (p, q) per 16 lanes (lane & 15 = 4 a + b: indices of the
// 4x4 blocks).  Gm / Gp: element (e, i; f, j) of the pair's G- / G+ block
// (rows 8 p + 4 e + i, columns 8 q + 4 f + j) at [(4 e + i) ld + 4 f + j]
// (complex FP64 or FP32).  The traces and block products run in F; the
// weight 1/(w_p w_q w_tau) and everything after it in FP64.  Returns the
// pair's weighted direct and exchange terms (zero unless ok) in every lane of
// the group and, with GRAD, writes the pair's adjoint blocks and their
// Hermitian partners into Hm / Hp (R x R, this tau; HT = double2, or
// uint32_t for BF16 pairs).
// The pair's h_p h_q (h = N_g / (g g) per walker pair) is read from the
// walker array, or passed in already loaded (PairH, for callers that load it
// ahead of the contraction).
struct PairH {
    double hp, hq;
};
__device__ inline double pair_h(const double *__restrict__ h, int p, int q) { return h[p] * h[q]; }
__device__ inline double pair_h(PairH h, int, int) { return h.hp * h.hq; }

// A pair's six adjoint block elements (lane (a, b): element [a][b] of H-(1,3),
// H-(2,4), H+(1,3), H+(2,4), H+(1,4), H+(2,3)) and their scale c (the last
// two take -c), for callers that store them themselves.
template <typename F>
struct AdjVals {
    cx<F> m13, m24, p13, p24, p14, p23;
    double cw;
};

template <bool GRAD, typename HT, typename F, typename GT, typename HV>
__device__ inline void contract_pair(const GT *Gm, const GT *Gp, int ld, int p, int q, bool ok, HV hinv, double wt,
                                     double cgrad, int R, double &dir, double &exc, HT *__restrict__ Hm,
                                     HT *__restrict__ Hp, AdjVals<F> *adj = nullptr) {
    const int lane = threadIdx.x & 63;
    const int a = (lane & 15) >> 2, b = lane & 3;
#define GB(G, e, f, i, j) to_cx<F>(G[(4 * (e) + (i)) * ld + 4 * (f) + (j)])
    cx<F> t1 = cmulc(GB(Gm, 0, 0, a, b), GB(Gp, 0, 0, a, b));
    cx<F> t2 = cmulc(GB(Gm, 1, 1, a, b), GB(Gp, 1, 1, a, b));
    cx<F> m1 = {0, 0}, m2 = {0, 0};
    for (int k = 0; k < 4; ++k) {
        m1 = cadd(m1, cmulc(GB(Gm, 0, 0, k, a), GB(Gp, 0, 1, k, b)));  // [G-(1,3)^H G+(1,4)]_{ab}
        m2 = cadd(m2, cmulc(GB(Gm, 1, 1, k, b), GB(Gp, 1, 0, k, a)));  // [G-(2,4)^H G+(2,3)]_{ba}
    }
    cx<F> xt = cmul(m1, m2);
    t1 = row16_sum(t1);
    t2 = row16_sum(t2);
    xt = row16_sum(xt);
    dir = exc = 0.0;
    if (ok) {
        const double W = pair_h(hinv, p, q) / wt;
        const cx<F> D = cmul(t1, t2);
        dir = -0.5 * (double)D.re * W;
        exc = 0.5 * (double)xt.re * W;
        if constexpr (GRAD) {
            // Adjoint of c Re(t1 t2 - X), c = cgrad W, with the stored blocks
            // A13 = G-(1,3), A24 = G-(2,4), P13 = G+(1,3), P14, P23, P24
            // (G-(3,1) = A13^H, G-(4,2) = A24^H):
            //   H-(1,3) = c (t2 P13 - P14 A24^H P23)   H-(2,4) = c (t1 P24 - P23 A13^H P14)
            //   H+(1,3) = c conj(t2) A13              H+(2,4) = c conj(t1) A24
            //   H+(1,4) = -c A13 P23^H A24            H+(2,3) = -c A24 P14^H A13
            // Lane (a, b) forms element [a][b] of each block.
            const double cw = cgrad * W;
            // The triple products as (X Y^H) Z: lane (a, b) forms [X Y^H]_{ab}
            // (four terms), then row a of it is gathered from lanes 4 a + l of
            // the pair's group for the product with Z.
            cx<F> x13 = {0, 0}, x24 = {0, 0}, x14 = {0, 0}, x23 = {0, 0};
            for (int k = 0; k < 4; ++k) {
                x13 = cadd(x13, cmul(GB(Gp, 0, 1, a, k), conjc(GB(Gm, 1, 1, b, k))));  // P14 A24^H
                x24 = cadd(x24, cmul(GB(Gp, 1, 0, a, k), conjc(GB(Gm, 0, 0, b, k))));  // P23 A13^H
                x14 = cadd(x14, cmul(GB(Gm, 0, 0, a, k), conjc(GB(Gp, 1, 0, b, k))));  // A13 P23^H
                x23 = cadd(x23, cmul(GB(Gm, 1, 1, a, k), conjc(GB(Gp, 0, 1, b, k))));  // A24 P14^H
            }
            cx<F> s13 = {0, 0}, s24 = {0, 0}, s14 = {0, 0}, s23 = {0, 0};
            auto gather = [&](auto lc) __attribute__((always_inline)) {  // element l of row a: lane 4 a + l
                constexpr int l = decltype(lc)::value;
                s13 = cadd(s13, cmul(quad_bcast<l>(x13), GB(Gp, 1, 0, l, b)));  // (P14 A24^H) P23
                s24 = cadd(s24, cmul(quad_bcast<l>(x24), GB(Gp, 0, 1, l, b)));  // (P23 A13^H) P14
                s14 = cadd(s14, cmul(quad_bcast<l>(x14), GB(Gm, 1, 1, l, b)));  // (A13 P23^H) A24
                s23 = cadd(s23, cmul(quad_bcast<l>(x23), GB(Gm, 0, 0, l, b)));  // (A24 P14^H) A13
            };
            gather(std::integral_constant<int, 0>());
            gather(std::integral_constant<int, 1>());
            gather(std::integral_constant<int, 2>());
            gather(std::integral_constant<int, 3>());
            const cx<F> p13 = GB(Gp, 0, 0, a, b), p24 = GB(Gp, 1, 1, a, b);
            const cx<F> a13 = GB(Gm, 0, 0, a, b), a24 = GB(Gm, 1, 1, a, b);
            const size_t r1 = 8 * p + a, r2 = 8 * p + 4 + a, c3 = 8 * q + b, c4 = 8 * q + 4 + b;
            // element (r, cc) = scale * v, its Hermitian partner (cc, r) = conj
            auto put = [&](HT *H, size_t r, size_t cc, cx<F> v, double scale) {
                if constexpr (std::is_same_v<HT, uint32_t>) {
                    // BF16 pairs: scaled in FP32 (BF16 keeps FP32's exponent range), rounded once
                    const float sc = (float)scale, re = (float)v.re * sc, im = (float)v.im * sc;
                    H[r * R + cc] = bf16_pair(re, im);
                    H[cc * R + r] = bf16_pair(re, -im);
                } else {
                    const double re = (double)v.re * scale, im = (double)v.im * scale;
                    h_store(H, r * R + cc, re, im);
                    h_store(H, cc * R + r, re, -im);
                }
            };
            const cx<F> h13 = csub(cmul(t2, p13), s13), h24 = csub(cmul(t1, p24), s24);
            const cx<F> g13 = cmul(conjc(t2), a13), g24 = cmul(conjc(t1), a24);
            if (adj) {
                *adj = AdjVals<F>{h13, h24, g13, g24, s14, s23, cw};
            } else {
                put(Hm, r1, c3, h13, cw);
                put(Hm, r2, c4, h24, cw);
                put(Hp, r1, c3, g13, cw);
                put(Hp, r2, c4, g24, cw);
                put(Hp, r1, c4, s14, -cw);
                put(Hp, r2, c3, s23, -cw);
            }
        }
    }
#undef GB
}

// ---------------------------------------------------------------------------
// Gaunt / Breit interaction (FP64).  g = sum_{mu nu} W_{mu nu}(r12) s_mu(1) s_nu(2)
// with s_0 = 1 and s_k = alpha_k (Eq. alpha), W_00 = 1/r, W_0k = W_k0 = 0,
// W_kl = -(delta_kl + c rhat_k rhat_l) / (2 r) (c = 1: both Breit terms of
// Sec. II, c = 0: the Gaunt term alone).  The 1/r12 and 1/r34 factors cancel
// against the pair weights as in the Coulomb case, leaving the dimensionless
// B_{mu nu} = r W_{mu nu} per walker pair.  With A13 = G-(1,3), A24 = G-(2,4),
// P_xy = G+(x,y) (G-(3,1) = A13^H, G-(4,2) = A24^H):
//   D = sum B12[mu nu] B34[rho sig] Tr[A13^H s_mu P13 s_rho] Tr[A24^H s_nu P24 s_sig]
//   X = sum B12[mu nu] B34[rho sig] Tr[A13^H s_mu P14 s_sig A24^H s_nu P23 s_rho]
// (s_rho acts at point 3, s_sig at point 4).
//
// On the components (L alpha, L beta, S alpha, S beta) every s_mu is
// monomial: row b holds its one non-zero entry ph(mu, b) in column
// b ^ sx(mu); alpha_x: 1; alpha_y: -i (b even), +i (b odd); alpha_z: +1
// (b even), -1 (b odd).  Products with s_mu are index permutations and phases.
__device__ __forceinline__ int sx(int mu) { return mu == 0 ? 0 : (mu == 3 ? 2 : 3); }
__device__ __forceinline__ cplx sph(int mu, int b, cplx z) {  // ph(mu, b) z
    if (mu == 2) return (b & 1) ? cplx{-z.im, z.re} : cplx{z.im, -z.re};
    if (mu == 3) return (b & 1) ? cplx{-z.re, -z.im} : z;
    return z;
}
// B[mu][nu] of one walker pair from its unit vector u (mu, nu may be runtime values)
__device__ __forceinline__ double bw(int mu, int nu, double ux, double uy, double uz, double c) {
    if (mu == 0 || nu == 0) return (mu == 0 && nu == 0) ? 1.0 : 0.0;
    const double um = mu == 1 ? ux : (mu == 2 ? uy : uz), un = nu == 1 ? ux : (nu == 2 ? uy : uz);
    return -0.5 * ((mu == nu ? 1.0 : 0.0) + c * um * un);
}

// Direct-part traces of one walker pair for lane (mu, rho) = (l16 >> 2, l16 & 3):
//   t1 = Tr[A13^H s_mu P13 s_rho],  t2 = Tr[A24^H s_mu P24 s_rho]
// (16 terms each; tiles as for contract_pair).
__device__ __attribute__((always_inline)) inline void breit_direct_traces(const cplx *Gm, const cplx *Gp, int ld,
                                                                           int l16, cplx &t1, cplx &t2) {
#define GB(G, e, f, i, j) G[(4 * (e) + (i)) * ld + 4 * (f) + (j)]
    const int mu = l16 >> 2, rho = l16 & 3, xm = sx(mu), xr = sx(rho);
    t1 = t2 = cplx{0, 0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            // Tr[A^H s_mu P s_rho] = sum_{a,b} conj(A[b][a]) ph(mu, b) P[b ^ xm][a ^ xr] ph(rho, a ^ xr)
            const cplx u1 = sph(mu, b, conjc(GB(Gm, 0, 0, b, a))), u2 = sph(mu, b, conjc(GB(Gm, 1, 1, b, a)));
            const cplx v1 = sph(rho, a ^ xr, GB(Gp, 0, 0, b ^ xm, a ^ xr));
            const cplx v2 = sph(rho, a ^ xr, GB(Gp, 1, 1, b ^ xm, a ^ xr));
            t1 = cadd(t1, cmul(u1, v1));
            t2 = cadd(t2, cmul(u2, v2));
        }
#undef GB
}

// One walker pair (p, q) per 16 lanes, tiles as for contract_pair (FP64
// complex); rhat [m_pad][4]: unit vectors of r1p - r2p; c: weight of the
// second Breit term.  Returns the weighted direct and exchange terms.
__device__ __attribute__((always_inline)) inline void contract_pair_breit(const cplx *Gm, const cplx *Gp, int ld, int p, int q, bool ok,
                                           const double *__restrict__ hinv, const double *__restrict__ rhat,
                                           double c, double wt, double &dir, double &exc) {
    const int lane = threadIdx.x & 63, l16 = lane & 15, grp = lane & ~15;
#define GB(G, e, f, i, j) G[(4 * (e) + (i)) * ld + 4 * (f) + (j)]
    const double ux = rhat[4 * p], uy = rhat[4 * p + 1], uz = rhat[4 * p + 2];
    const double vx = rhat[4 * q], vy = rhat[4 * q + 1], vz = rhat[4 * q + 2];

    // direct: lane (mu, rho) forms T1[mu][rho] and T2[mu][rho], then
    // T1[mu][rho] sum_{nu, sig} B12[mu][nu] B34[rho][sig] T2[nu][sig]
    cplx dterm;
    {
        const int mu = l16 >> 2, rho = l16 & 3;
        cplx t1, t2;
        breit_direct_traces(Gm, Gp, ld, l16, t1, t2);
        // T2 gathered from lane 4 nu + sig
        cplx acc = {0, 0};
#pragma unroll
        for (int nu = 0; nu < 4; ++nu)
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                const cplx t = shfl_c(t2, grp | (4 * nu + sg));
                const double w = bw(mu, nu, ux, uy, uz, c) * bw(rho, sg, vx, vy, vz, c);
                acc = {acc.re + w * t.re, acc.im + w * t.im};
            }
        dterm = cmul(t1, acc);
    }
    // exchange: lane (a, b) = (l16 >> 2, l16 & 3) forms element [a][b] of
    //   L_{mu sig} = A13^H s_mu P14 s_sig  and element [b][a] of  R_{nu rho} = A24^H s_nu P23 s_rho,
    //   L_{mu sig}[a][b] = ph(sig, b ^ x_sig) sum_k conj(A13[k ^ x_mu][a]) ph(mu, k ^ x_mu) P14[k][b ^ x_sig]
    //   R_{nu rho}[b][a] = ph(rho, a ^ x_rho) sum_k conj(A24[k ^ x_nu][b]) ph(nu, k ^ x_nu) P23[k][a ^ x_rho]
    // and sums L_{mu sig}[a][b] Rw[mu][sig] with Rw[mu][sig] = sum B12[mu][nu] B34[rho][sig] R_{nu rho}[b][a].
    cplx xterm = {0, 0};
    {
        const int a = l16 >> 2, b = l16 & 3;
        cplx S[4][4];  // S[nu][sig] = sum_rho B34[rho][sig] R_{nu rho}
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            cplx Rr[4];
#pragma unroll
            for (int rho = 0; rho < 4; ++rho) {
                const int cc = a ^ sx(rho);
                cplx z = {0, 0};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    z = cadd(z, cmul(sph(nu, k ^ sx(nu), conjc(GB(Gm, 1, 1, k ^ sx(nu), b))), GB(Gp, 1, 0, k, cc)));
                Rr[rho] = sph(rho, cc, z);
            }
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                cplx t = {0, 0};
#pragma unroll
                for (int rho = 0; rho < 4; ++rho) {
                    const double w = bw(rho, sg, vx, vy, vz, c);
                    t = {t.re + w * Rr[rho].re, t.im + w * Rr[rho].im};
                }
                S[nu][sg] = t;
            }
        }
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int sg = 0; sg < 4; ++sg) {
                cplx rw = {0, 0};
#pragma unroll
                for (int nu = 0; nu < 4; ++nu) {
                    const double w = bw(mu, nu, ux, uy, uz, c);
                    rw = {rw.re + w * S[nu][sg].re, rw.im + w * S[nu][sg].im};
                }
                const int cc = b ^ sx(sg);
                cplx y = {0, 0};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    y = cadd(y, cmul(sph(mu, k ^ sx(mu), conjc(GB(Gm, 0, 0, k ^ sx(mu), a))), GB(Gp, 0, 1, k, cc)));
                xterm = cadd(xterm, cmul(sph(sg, cc, y), rw));
            }
    }
    for (int mask = 8; mask >= 1; mask >>= 1) {
        dterm = cadd(dterm, shfl_xor_c(dterm, mask));
        xterm = cadd(xterm, shfl_xor_c(xterm, mask));
    }
    dir = exc = 0.0;
    if (ok) {
        const double W = hinv[p] * hinv[q] / wt;
        dir = -0.5 * dterm.re * W;
        exc = 0.5 * xterm.re * W;
    }
#undef GB
}

// contract_pairs with the Gaunt / Breit interaction (FP64).
__device__ __attribute__((always_inline)) inline void contract_pairs_breit(const cplx *Gm, const cplx *Gp, int PT, int QT, int m,
                                            const double *__restrict__ hinv, const double *__restrict__ rhat,
                                            double c, double wt, double *__restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wp = wave >> 1, wq = wave & 1;
    const int pi = lane >> 4, pp = pi >> 1, qq = pi & 1;
    const int p = kTileWalkers * PT + 2 * wp + pp, q = kTileWalkers * QT + 2 * wq + qq;
    double dir, exc;
    contract_pair_breit(Gm + 8 * pp * 16 + 8 * qq, Gp + 8 * pp * 16 + 8 * qq, 16, p, q, p < q && q < m, hinv, rhat,
                        c, wt, dir, exc);
    const double d0 = __shfl(dir, 0, 64), d1 = __shfl(dir, 16, 64), d2 = __shfl(dir, 32, 64),
                 d3 = __shfl(dir, 48, 64);
    const double x0 = __shfl(exc, 0, 64), x1 = __shfl(exc, 16, 64), x2 = __shfl(exc, 32, 64),
                 x3 = __shfl(exc, 48, 64);
    if (lane == 0) {
        out[0] = ((d0 + d1) + d2) + d3;
        out[1] = ((x0 + x1) + x2) + x3;
    }
}

// ph(mu, b) as a power of i (sph multiplies by i^qph)
__device__ __forceinline__ int qph(int mu, int b) { return mu == 2 ? ((b & 1) ? 1 : 3) : (mu == 3 ? ((b & 1) ? 2 : 0) : 0); }
// i^q z
__device__ __forceinline__ cplx qrot(cplx z, int q) {
    const cplx s = (q & 1) ? cplx{-z.im, z.re} : z;
    return (q & 2) ? cplx{-s.re, -s.im} : s;
}

// Sum over the 16 lanes of a row of the 16 values v[e], lane l16 of the row
// ending with the sum of v[l16]: four halving steps, each lane keeping the
// half of its values whose index bit matches its own lane bit (3, 2, 1, 0)
// and adding the partner's copy of that half (partners: row_ror:8,
// row_half_mirror, xor 2, xor 1 -- each flips the step's bit and none of the
// bits above it).
__device__ inline cplx row16_reduce_scatter(const cplx (&v)[16], int l16) {
    const bool b3 = l16 & 8, b2 = l16 & 4, b1 = l16 & 2, b0 = l16 & 1;
    cplx r8[8], r4[4], r2[2];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const cplx send = b3 ? v[n] : v[n + 8], keep = b3 ? v[n + 8] : v[n];
        r8[n] = cadd(keep, dpp_c<0x128>(send));
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const cplx send = b2 ? r8[n] : r8[n + 4], keep = b2 ? r8[n + 4] : r8[n];
        r4[n] = cadd(keep, dpp_c<0x141>(send));
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const cplx send = b1 ? r4[n] : r4[n + 2], keep = b1 ? r4[n + 2] : r4[n];
        r2[n] = cadd(keep, dpp_c<0x4E>(send));
    }
    const cplx send = b0 ? r2[0] : r2[1], keep = b0 ? r2[1] : r2[0];
    return cadd(keep, dpp_c<0xB1>(send));
}

// Exchange blocks of the Breit adjoint.  Each has the form
//   Y = sum_{al, be} s_al L K[al][be] Rm s_be,
//   K[al][be] = sum_{ga, de} B12[al][ga] B34[be][de] s_de M s_ga = S2(be) M S1(al),
//   S1(al) = sum_ga B12[al][ga] s_ga,  S2(be) = sum_de B34[be][de] s_de
// (L, M, Rm: 4x4 blocks read through accessors; b1[ga] = B12[al][ga] and
// b2[de] = B34[be][de] of this lane).  Lane (al, be) = (l16 >> 2, l16 & 3) of
// the pair's group forms its term (s_al L) K (Rm s_be) -- the alpha factors
// as permuted reads and phases, every register index a compile-time one --
// and the 16 terms are summed, lane (a, b) keeping entry [a][b].
template <typename FL, typename FM, typename FR>
__device__ inline cplx breit_xblock(FL L, FM M, FR Rm, int l16, const double (&b1)[4], const double (&b2)[4]) {
    const int al = l16 >> 2, be = l16 & 3, xa = sx(al), xb = sx(be);
    cplx N[4][4];  // M S1: (M s_ga)[r][l] = M[r][l ^ x_ga] ph(ga, l ^ x_ga)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            cplx z = {0, 0};
#pragma unroll
            for (int ga = 0; ga < 4; ++ga) {
                const cplx t = sph(ga, l ^ sx(ga), M(r, l ^ sx(ga)));
                z = {z.re + b1[ga] * t.re, z.im + b1[ga] * t.im};
            }
            N[r][l] = z;
        }
    cplx K[4][4];  // S2 N: (s_de N)[k][l] = ph(de, k) N[k ^ x_de][l]
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            cplx z = {0, 0};
#pragma unroll
            for (int de = 0; de < 4; ++de) {
                const cplx t = sph(de, k, N[k ^ sx(de)][l]);
                z = {z.re + b2[de] * t.re, z.im + b2[de] * t.im};
            }
            K[k][l] = z;
        }
    cplx LK[4][4];  // L[i ^ x_al][.] K; the phase ph(al, i) of s_al goes on the result
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            cplx z = {0, 0};
#pragma unroll
            for (int k = 0; k < 4; ++k) z = cadd(z, cmul(L(i ^ xa, k), K[k][l]));
            LK[i][l] = z;
        }
    cplx y[16];  // (Rm s_be)[l][j] = Rm[l][j ^ x_be] ph(be, j ^ x_be)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cplx z = {0, 0};
#pragma unroll
            for (int l = 0; l < 4; ++l) z = cadd(z, cmul(LK[i][l], Rm(l, j ^ xb)));
            y[4 * i + j] = qrot(z, qph(al, i) + qph(be, j ^ xb));
        }
    return row16_reduce_scatter(y, l16);
}

// Adjoint of one walker pair's Gaunt / Breit terms (16 lanes, tiles as for
// contract_pair): writes the pair's six 4x4 blocks of H- and H+ (FP64) and
// their Hermitian partners, as contract_pair<true> does for the Coulomb
// interaction; ok = false writes nothing.  With cw = cgrad W:
//   H-(1,3) = cw (sum_{mu rho} U[mu][rho] s_mu P13 s_rho - X1)
//   H-(2,4) = cw (sum_{nu sig} V[nu][sig] s_nu P24 s_sig - X2)
//   H+(1,3) = cw sum conj(U[mu][rho]) s_mu A13 s_rho,  H+(2,4) = cw sum conj(V[nu][sig]) s_nu A24 s_sig
//   H+(1,4) = -cw X3,  H+(2,3) = -cw X4
// with U[mu][rho] = sum B12[mu][nu] B34[rho][sig] T2[nu][sig] and
// V[nu][sig] = sum B12[mu][nu] B34[rho][sig] T1[mu][rho] (T1, T2: the direct
// traces), and the exchange blocks (breit_xblock)
//   X1 = sum s_mu P14 [sum B12[mu nu] B34[rho sig] s_sig A24^H s_nu] P23 s_rho,
//   X2 = sum s_nu P23 [sum B12[mu nu] B34[rho sig] s_rho A13^H s_mu] P14 s_sig,
//   X3 = sum s_mu A13 [sum B12[mu nu] B34[rho sig] s_rho P23^H s_nu] A24 s_sig,
//   X4 = sum s_nu A24 [sum B12[mu nu] B34[rho sig] s_sig P14^H s_mu] A13 s_rho.
// HT: double2 (FP64 blocks) or uint32_t (BF16 pairs, rounded once from FP64).
template <typename HT>
__device__ inline void breit_adjoint_pair(const cplx *Gm, const cplx *Gp, int ld, int p, int q, bool ok,
                                          const double *__restrict__ hinv, const double *__restrict__ rhat, double c,
                                          double wt, double cgrad, int R, HT *__restrict__ Hm,
                                          HT *__restrict__ Hp) {
    if (!ok) return;  // ok is the same in all 16 lanes of the pair
    const int lane = threadIdx.x & 63, l16 = lane & 15, grp = lane & ~15;
    const int a = l16 >> 2, b = l16 & 3;
#define GB(G, e, f, i, j) G[(4 * (e) + (i)) * ld + 4 * (f) + (j)]
    const double ux = rhat[4 * p], uy = rhat[4 * p + 1], uz = rhat[4 * p + 2];
    const double vx = rhat[4 * q], vy = rhat[4 * q + 1], vz = rhat[4 * q + 2];
    double b1[4], b2[4];  // B12[a][.], B34[b][.] of this lane
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        b1[g] = bw(a, g, ux, uy, uz, c);
        b2[g] = bw(b, g, vx, vy, vz, c);
    }
    cplx t1, t2;
    breit_direct_traces(Gm, Gp, ld, l16, t1, t2);
    cplx U = {0, 0}, V = {0, 0};  // lane (a, b): U[a][b], V[a][b]
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double w = b1[e] * b2[f];
            const cplx s2 = shfl_c(t2, grp | (4 * e + f)), s1 = shfl_c(t1, grp | (4 * e + f));
            U = {U.re + w * s2.re, U.im + w * s2.im};
            V = {V.re + w * s1.re, V.im + w * s1.im};
        }
    const double cw = cgrad * hinv[p] * hinv[q] / wt;
    cplx h13m = {0, 0}, h24m = {0, 0}, h13p = {0, 0}, h24p = {0, 0};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int rho = 0; rho < 4; ++rho) {
            const cplx Um = shfl_c(U, grp | (4 * mu + rho)), Vm = shfl_c(V, grp | (4 * mu + rho));
            const int r = a ^ sx(mu), cc = b ^ sx(rho);
            // (s_mu Z s_rho)[a][b] = ph(mu, a) Z[a ^ x_mu][b ^ x_rho] ph(rho, b ^ x_rho)
            const int qp = qph(mu, a) + qph(rho, cc);
            h13m = cadd(h13m, cmul(Um, qrot(GB(Gp, 0, 0, r, cc), qp)));
            h13p = cadd(h13p, cmul(conjc(Um), qrot(GB(Gm, 0, 0, r, cc), qp)));
            h24m = cadd(h24m, cmul(Vm, qrot(GB(Gp, 1, 1, r, cc), qp)));
            h24p = cadd(h24p, cmul(conjc(Vm), qrot(GB(Gm, 1, 1, r, cc), qp)));
        }
    const size_t r1 = 8 * p + a, r2 = 8 * p + 4 + a, c3 = 8 * q + b, c4 = 8 * q + 4 + b;
    auto put = [&](HT *H, size_t r, size_t cc, cplx v, double scale) {  // and the Hermitian partner
        h_store(H, r * R + cc, v.re * scale, v.im * scale);
        h_store(H, cc * R + r, v.re * scale, -v.im * scale);
    };
    put(Hp, r1, c3, h13p, cw);
    put(Hp, r2, c4, h24p, cw);
    // the four exchange blocks in one loop (not unrolled: one block's registers at a time);
    // L and Rm are plain 4x4 blocks, M a conjugate-transposed one:
    //   X1: (P14, A24, P23)  X2: (P23, A13, P14)  X3: (A13, P23, A24)  X4: (A24, P14, A13)
#pragma nounroll
    for (int x = 0; x < 4; ++x) {
        const cplx *Lb = x == 0 ? &GB(Gp, 0, 1, 0, 0) : x == 1 ? &GB(Gp, 1, 0, 0, 0) : x == 2 ? &GB(Gm, 0, 0, 0, 0)
                                                                                        : &GB(Gm, 1, 1, 0, 0);
        const cplx *Mb = x == 0 ? &GB(Gm, 1, 1, 0, 0) : x == 1 ? &GB(Gm, 0, 0, 0, 0) : x == 2 ? &GB(Gp, 1, 0, 0, 0)
                                                                                        : &GB(Gp, 0, 1, 0, 0);
        const cplx *Rb = x == 0 ? &GB(Gp, 1, 0, 0, 0) : x == 1 ? &GB(Gp, 0, 1, 0, 0) : x == 2 ? &GB(Gm, 1, 1, 0, 0)
                                                                                        : &GB(Gm, 0, 0, 0, 0);
        const cplx y = breit_xblock([&](int i, int j) { return Lb[i * ld + j]; },
                                    [&](int i, int j) { return conjc(Mb[j * ld + i]); },
                                    [&](int i, int j) { return Rb[i * ld + j]; }, l16, b1, b2);
        // X1 -> H-(1,3), X2 -> H-(2,4) (with the direct sums), X3 -> H+(1,4), X4 -> H+(2,3)
        const cplx h = x == 0 ? csub(h13m, y) : x == 1 ? csub(h24m, y) : y;
        put(x < 2 ? Hm : Hp, (x & 1) ? r2 : r1, x == 0 || x == 3 ? c3 : c4, h, x < 2 ? cw : -cw);
    }
#undef GB
}

// One wave, one tau sample.  Gm / Gp: this wave's 16x16 sub-tiles of G- and
// G+ (complex FP64, row-major, rows 8 pp + 4 e + i of block-tile row PT,
// columns 8 qq + 4 f + j of block-tile column QT; the wave's sub-tile origin
// is (wp, wq) = (wave >> 1, wave & 1)).  16 lanes per walker pair: (pp, qq) =
// walker offsets in the sub-tile.  Writes the wave's direct and exchange
// sums to out[0], out[1] and, with GRAD, the pairs' adjoint blocks.
template <bool GRAD, typename HT, typename F = double>
__device__ inline void contract_pairs(const cplx *Gm, const cplx *Gp, int PT, int QT, int m,
                                      const double *__restrict__ hinv, double wt, double cgrad, int R,
                                      double *__restrict__ out, HT *__restrict__ Hm, HT *__restrict__ Hp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wp = wave >> 1, wq = wave & 1;
    const int pi = lane >> 4, pp = pi >> 1, qq = pi & 1;
    const int p = kTileWalkers * PT + 2 * wp + pp, q = kTileWalkers * QT + 2 * wq + qq;
    double dir, exc;
    contract_pair<GRAD, HT, F>(Gm + 8 * pp * 16 + 8 * qq, Gp + 8 * pp * 16 + 8 * qq, 16, p, q, p < q && q < m,
                                    hinv, wt, cgrad, R, dir, exc, Hm, Hp);
    // pairs of this wave summed in a fixed order (lanes 0, 16, 32, 48)
    const double d0 = lane_value(dir, 0), d1 = lane_value(dir, 16), d2 = lane_value(dir, 32),
                 d3 = lane_value(dir, 48);
    const double x0 = lane_value(exc, 0), x1 = lane_value(exc, 16), x2 = lane_value(exc, 32),
                 x3 = lane_value(exc, 48);
    if (lane == 0) {
        out[0] = ((d0 + d1) + d2) + d3;
        out[1] = ((x0 + x1) + x2) + x3;
    }
}
