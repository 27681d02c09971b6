// Green's functions and pair contraction of the MC-MP2 integrand (Sec. III
// of the paper, the G+ / G- definitions and Eq. redundant), FP64.
//
// For tau sample t the operands are the spinor values psi[k][r] scaled by
//   s_k = exp(+eps_k tau)  (occupied, G-)   or   exp(-eps_k tau)  (virtual, G+),
// and the Green's functions over all 8m x 8m rows are
//   G(x, y) = sum_k s_k psi[k][x] conj(psi[k][y]).
// Only the 8x8 blocks of walker pairs p < q enter the estimator, and
// G(y, x) = G(x, y)^dagger, so the kernel walks the upper triangle of
// 16x16-row tiles (2 walker pairs per tile side).  One wave owns one tile
// pair and computes both G- and G+ for it on FP64 MFMA, complex as real
// pairs: with psi_x = a + ib and psi_y = c + id,
//   Re G += a c + b d,   Im G += b c - a d.
// The tile never leaves the chip: the wave stages it in LDS and contracts
// the (up to) four walker pairs it covers,
//   D = Tr[G-(3,1) G+(1,3)] Tr[G-(4,2) G+(2,4)],
//   X = Tr[G-(3,1) G+(1,4) G-(4,2) G+(2,3)],
// (1 = r1p, 2 = r2p, 3 = r1q, 4 = r2q; G(3,1) = G(1,3)^dagger), and weights
// each pair by N_g^2 / (g(1) g(2) g(3) g(4) w(tau)) -- the 1/(r12 r34) of the
// integrand cancels the 1/r of the two pair weights.  Per tile pair it
// writes the direct part -Re(D)/2 and the exchange part +Re(X)/2; a second
// kernel reduces them with compensated (Neumaier) summation in a fixed order.
#include "internal.hpp"

namespace {

__global__ void tau_prep_kernel(const double *__restrict__ tau, const double *__restrict__ eps, int n_tau, int nsp,
                                int no, double lambda, double *__restrict__ scale, double *__restrict__ wtau) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int t = blockIdx.y;
    if (t >= n_tau || k >= nsp) return;
    double tv = tau[t];
    scale[(size_t)t * nsp + k] = k < no ? exp(eps[k] * tv) : exp(-eps[k] * tv);
    if (k == 0) wtau[t] = lambda * exp(-lambda * tv);
}

struct cplx {
    double re, im;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cmulc(cplx a, cplx b) {  // conj(a) * b
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx shfl_xor_c(cplx a, int mask) {
    return {__shfl_xor(a.re, mask, 64), __shfl_xor(a.im, mask, 64)};
}

// Accumulate sum_k s_k psi[k][rp + i] conj(psi[k][rq + j]) for k in [k_lo, k_hi).
__device__ inline void green_tile(const double2 *__restrict__ psi, const double *__restrict__ sc, int R, int rp,
                                  int rq, int k_lo, int k_hi, int li, int lk, d4v &acc_re, d4v &acc_im) {
    for (int k0 = k_lo; k0 < k_hi; k0 += 4) {
        const int k = k0 + lk;
        double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
        if (k < k_hi) {
            const double s = sc[k];
            const double2 x = psi[(size_t)k * R + rp + li];
            const double2 y = psi[(size_t)k * R + rq + li];
            a = x.x * s;
            b = x.y * s;
            c = y.x;
            d = y.y;
        }
        acc_re = __builtin_amdgcn_mfma_f64_16x16x4f64(a, c, acc_re, 0, 0, 0);
        acc_re = __builtin_amdgcn_mfma_f64_16x16x4f64(b, d, acc_re, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f64_16x16x4f64(b, c, acc_im, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, d, acc_im, 0, 0, 0);
    }
}

__global__ __launch_bounds__(256) void green_contract_kernel(const double *__restrict__ psi_, const double *__restrict__ scale,
                                                             const double *__restrict__ wtau,
                                                             const double *__restrict__ hinv,
                                                             const int *__restrict__ tiles, int n_tp, int R, int no,
                                                             int nsp, int m, double *__restrict__ partial) {
    __shared__ cplx lds[4][2][256];
    const double2 *psi = reinterpret_cast<const double2 *>(psi_);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tp = blockIdx.x * 4 + wave;
    const int t = blockIdx.y;
    const bool active = tp < n_tp;
    const int li = lane & 15, lk = lane >> 4;
    const double *sc = scale + (size_t)t * nsp;

    int P = 0, Q = 0;
    if (active) {
        P = tiles[2 * tp];
        Q = tiles[2 * tp + 1];
        const int rp = 16 * P, rq = 16 * Q;
        d4v gm_re = {0, 0, 0, 0}, gm_im = {0, 0, 0, 0}, gp_re = {0, 0, 0, 0}, gp_im = {0, 0, 0, 0};
        green_tile(psi, sc, R, rp, rq, 0, no, li, lk, gm_re, gm_im);
        green_tile(psi, sc, R, rp, rq, no, nsp, li, lk, gp_re, gp_im);
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * v + lk;  // MFMA f64 result row of element v
            lds[wave][0][i * 16 + li] = {gm_re[v], gm_im[v]};
            lds[wave][1][i * 16 + li] = {gp_re[v], gp_im[v]};
        }
    }
    __syncthreads();
    if (!active) return;

    // 16 lanes per walker pair: (pp, qq) = walker offsets in the tiles,
    // (a, b) = 4x4 matrix indices of this lane.
    const int pi = lane >> 4, pp = pi >> 1, qq = pi & 1;
    const int a = (lane & 15) >> 2, b = lane & 3;
    const cplx *Gm = lds[wave][0];
    const cplx *Gp = lds[wave][1];
    // block (e, e') of the pair: rows 8 pp + 4 e + i, cols 8 qq + 4 e' + j
#define GB(G, e, f, i, j) G[(8 * pp + 4 * (e) + (i)) * 16 + 8 * qq + 4 * (f) + (j)]
    cplx t1 = cmulc(GB(Gm, 0, 0, a, b), GB(Gp, 0, 0, a, b));
    cplx t2 = cmulc(GB(Gm, 1, 1, a, b), GB(Gp, 1, 1, a, b));
    cplx m1 = {0.0, 0.0}, m2 = {0.0, 0.0};
    for (int k = 0; k < 4; ++k) {
        m1 = cadd(m1, cmulc(GB(Gm, 0, 0, k, a), GB(Gp, 0, 1, k, b)));  // [G-(1,3)^H G+(1,4)]_{ab}
        m2 = cadd(m2, cmulc(GB(Gm, 1, 1, k, b), GB(Gp, 1, 0, k, a)));  // [G-(2,4)^H G+(2,3)]_{ba}
    }
#undef GB
    cplx xt = cmul(m1, m2);
    for (int mask = 8; mask >= 1; mask >>= 1) {
        t1 = cadd(t1, shfl_xor_c(t1, mask));
        t2 = cadd(t2, shfl_xor_c(t2, mask));
        xt = cadd(xt, shfl_xor_c(xt, mask));
    }
    const int p = kTileWalkers * P + pp, q = kTileWalkers * Q + qq;
    double dir = 0.0, exc = 0.0;
    if (p < q && q < m) {
        const double W = hinv[p] * hinv[q] / wtau[t];
        const cplx D = cmul(t1, t2);
        dir = -0.5 * D.re * W;
        exc = 0.5 * xt.re * W;
    }
    // pairs of this wave summed in a fixed order (lanes 0, 16, 32, 48)
    double d0 = __shfl(dir, 0, 64), d1 = __shfl(dir, 16, 64), d2 = __shfl(dir, 32, 64), d3 = __shfl(dir, 48, 64);
    double x0 = __shfl(exc, 0, 64), x1 = __shfl(exc, 16, 64), x2 = __shfl(exc, 32, 64), x3 = __shfl(exc, 48, 64);
    if (lane == 0) {
        double *out = partial + ((size_t)t * n_tp + tp) * 2;
        out[0] = ((d0 + d1) + d2) + d3;
        out[1] = ((x0 + x1) + x2) + x3;
    }
}

// Neumaier (improved Kahan) summation: s + c carries the running total.
__device__ inline void neumaier_add(double &s, double &c, double x) {
    double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// One block per tau: per-thread compensated sums over a fixed stride, then a
// fixed-order compensated sum of the 256 thread totals by thread 0.
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial, int n_tp, double inv_pairs,
                                                     double *__restrict__ e2_out) {
    __shared__ double sd[256], sx[256];
    const int t = blockIdx.x;
    const double *src = partial + (size_t)t * n_tp * 2;
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    for (int i = threadIdx.x; i < n_tp; i += 256) {
        neumaier_add(s0, c0, src[2 * i]);
        neumaier_add(s1, c1, src[2 * i + 1]);
    }
    sd[threadIdx.x] = s0 + c0;
    sx[threadIdx.x] = s1 + c1;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0;
        for (int i = 0; i < 256; ++i) {
            neumaier_add(a0, b0, sd[i]);
            neumaier_add(a1, b1, sx[i]);
        }
        const double d = (a0 + b0) * inv_pairs, x = (a1 + b1) * inv_pairs;
        e2_out[3 * t] = d;
        e2_out[3 * t + 1] = x;
        e2_out[3 * t + 2] = d + x;
    }
}

}  // namespace

hipError_t launch_tau_prep(const mcmp2_ctx *c, const double *tau, int n_tau) {
    dim3 grid((c->nsp + 255) / 256, n_tau);
    tau_prep_kernel<<<grid, 256, 0, c->stream>>>(tau, c->eps, n_tau, c->nsp, c->no, c->lambda, c->scale, c->wtau);
    return hipGetLastError();
}

hipError_t launch_green_contract(const mcmp2_ctx *c, int n_tau) {
    dim3 grid((c->n_tp + 3) / 4, n_tau);
    green_contract_kernel<<<grid, 256, 0, c->stream>>>(c->psi, c->scale, c->wtau, c->hinv, c->tiles, c->n_tp, c->R,
                                                       c->no, c->nsp, c->m, c->partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const mcmp2_ctx *c, int n_tau, double *e2_out) {
    const double pairs = 0.5 * (double)c->m * (double)(c->m - 1);
    reduce_kernel<<<n_tau, 256, 0, c->stream>>>(c->partial, c->n_tp, 1.0 / pairs, e2_out);
    return hipGetLastError();
}
