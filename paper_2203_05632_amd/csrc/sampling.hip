// Samplers and weights of the MC-MP2 estimator (Sec. III of the paper):
// electron-pair weight w(r1, r2) = g(r1) g(r2) / (N_g r12) with g of
// Eq. basisSet, Metropolis moves of the walker pairs, and inverse-CDF
// sampling of tau from w(tau) = lambda exp(-lambda tau).
//
// Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
// (key0, key1) and counter (step, index, purpose, 0).
//
// Floating-point contraction is disabled in this file so that the walker
// positions r + delta (2u - 1) are reproduced bit for bit by any IEEE
// evaluation of the same expression.
#pragma clang fp contract(off)

#include <algorithm>

#include "internal.hpp"

namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

struct u64x4 {
    uint64_t x[4];
};

__device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                      uint64_t k1) {
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kW0;
            k1 += kW1;
        }
        uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
        uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
        uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    return {{x0, x1, x2, x3}};
}

__device__ inline double to_unit(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }

__device__ inline double dist(const double *a, const double *b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// w[p] = g(r1) g(r2) / (N_g r12) and hinv[p] = N_g / (g(r1) g(r2)).
__global__ void walker_weights_kernel(const double *__restrict__ walkers, int m, const double *__restrict__ nuc,
                                      const double *__restrict__ gpar, int n_nuc, double Ng, double *w,
                                      double *hinv) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const double *r1 = walkers + 6 * p, *r2 = r1 + 3;
    double g1 = g_value(r1[0], r1[1], r1[2], nuc, gpar, n_nuc);
    double g2 = g_value(r2[0], r2[1], r2[2], nuc, gpar, n_nuc);
    if (w) w[p] = (g1 * g2) / (Ng * dist(r1, r2));
    if (hinv) hinv[p] = Ng / (g1 * g2);
}

__device__ inline void metropolis_pair(int p, double *__restrict__ walkers, double *__restrict__ w,
                                       const double *__restrict__ nuc, const double *__restrict__ gpar, int n_nuc,
                                       double Ng, uint64_t key0, uint64_t key1, uint64_t step, double delta,
                                       int32_t *n_acc) {
    u64x4 a = philox4x64_10(step, (uint64_t)p, 0, 0, key0, key1);
    u64x4 b = philox4x64_10(step, (uint64_t)p, 1, 0, key0, key1);
    double u[6] = {to_unit(a.x[0]), to_unit(a.x[1]), to_unit(a.x[2]),
                   to_unit(a.x[3]), to_unit(b.x[0]), to_unit(b.x[1])};
    double trial[6];
    for (int i = 0; i < 6; ++i) trial[i] = walkers[6 * p + i] + delta * (2.0 * u[i] - 1.0);
    double g1 = g_value(trial[0], trial[1], trial[2], nuc, gpar, n_nuc);
    double g2 = g_value(trial[3], trial[4], trial[5], nuc, gpar, n_nuc);
    double wt = (g1 * g2) / (Ng * dist(trial, trial + 3));
    if (to_unit(b.x[2]) < wt / w[p]) {
        for (int i = 0; i < 6; ++i) walkers[6 * p + i] = trial[i];
        w[p] = wt;
        if (n_acc) atomicAdd(n_acc, 1);
    }
}

__device__ inline double tau_value(int t, uint64_t key0, uint64_t key1, uint64_t step, double lambda) {
    u64x4 a = philox4x64_10(step, (uint64_t)t, 2, 0, key0, key1);
    return -log(1.0 - to_unit(a.x[0])) / lambda;
}

__global__ void metropolis_kernel(double *__restrict__ walkers, double *__restrict__ w, int m,
                                  const double *__restrict__ nuc, const double *__restrict__ gpar, int n_nuc,
                                  double Ng, uint64_t key0, uint64_t key1, uint64_t step, double delta,
                                  int32_t *n_acc) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) metropolis_pair(p, walkers, w, nuc, gpar, n_nuc, Ng, key0, key1, step, delta, n_acc);
}

__global__ void sample_tau_kernel(uint64_t key0, uint64_t key1, uint64_t step, int n_tau, double lambda,
                                  double *tau) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tau) tau[t] = tau_value(t, key0, key1, step, lambda);
}

// Both samplers of one MC step in a single launch: threads [0, m) move the
// walker pairs, threads [m, m + n_tau) draw the tau samples.
__global__ void advance_kernel(double *__restrict__ walkers, double *__restrict__ w, int m,
                               const double *__restrict__ nuc, const double *__restrict__ gpar, int n_nuc, double Ng,
                               uint64_t key0, uint64_t key1, uint64_t step, double delta, int32_t *n_acc, int n_tau,
                               double lambda, double *tau) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        metropolis_pair(i, walkers, w, nuc, gpar, n_nuc, Ng, key0, key1, step, delta, n_acc);
    else if (i < m + n_tau)
        tau[i - m] = tau_value(i - m, key0, key1, step, lambda);
}

// Compensated accumulation with neumaier() (internal.hpp).
__global__ void accumulate_kernel(const double *__restrict__ src, double *__restrict__ sum, double *__restrict__ comp,
                                  int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = sum[i], c = comp[i];
        neumaier(s, c, src[i]);
        comp[i] = c;
        sum[i] = s;
    }
}

// The same steps on 16-byte aligned arrays, two doubles per access; the
// last element of an odd n goes to thread 0.
typedef double d2x __attribute__((ext_vector_type(2)));
__global__ void accumulate2_kernel(const double *__restrict__ src, double *__restrict__ sum,
                                   double *__restrict__ comp, int64_t n) {
    const int64_t n2 = n / 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const d2x x = reinterpret_cast<const d2x *>(src)[i];
        d2x s = reinterpret_cast<const d2x *>(sum)[i], c = reinterpret_cast<const d2x *>(comp)[i];
        double s0 = s[0], s1 = s[1], c0 = c[0], c1 = c[1];
        neumaier(s0, c0, x[0]);
        neumaier(s1, c1, x[1]);
        reinterpret_cast<d2x *>(comp)[i] = d2x{c0, c1};
        reinterpret_cast<d2x *>(sum)[i] = d2x{s0, s1};
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = sum[n - 1], c = comp[n - 1];
        neumaier(s, c, src[n - 1]);
        comp[n - 1] = c;
        sum[n - 1] = s;
    }
}

}  // namespace

hipError_t launch_accumulate(const mcmp2_ctx *c, const double *src, double *sum, double *comp, int64_t n) {
    if (n == 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(sum) |
                           reinterpret_cast<uintptr_t>(comp)) & 15) == 0;
    if (aligned) {
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n / 2 + 255) / 256, 4096));
        accumulate2_kernel<<<(int)blocks, 256, 0, c->stream>>>(src, sum, comp, n);
    } else {
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
        accumulate_kernel<<<(int)blocks, 256, 0, c->stream>>>(src, sum, comp, n);
    }
    return hipGetLastError();
}

hipError_t launch_walker_weights(const mcmp2_ctx *c, const double *walkers, double *w, double *hinv) {
    int nb = (c->m + 63) / 64;
    walker_weights_kernel<<<nb, 64, 0, c->stream>>>(walkers, c->m, c->nuc, c->gpar, c->n_nuc, c->Ng, w, hinv);
    return hipGetLastError();
}

hipError_t launch_metropolis(const mcmp2_ctx *c, double *walkers, double *w, uint64_t key0, uint64_t key1,
                             uint64_t step, double delta, int32_t *n_acc) {
    int nb = (c->m + 63) / 64;
    metropolis_kernel<<<nb, 64, 0, c->stream>>>(walkers, w, c->m, c->nuc, c->gpar, c->n_nuc, c->Ng, key0, key1,
                                                step, delta, n_acc);
    return hipGetLastError();
}

hipError_t launch_advance(const mcmp2_ctx *c, double *walkers, double *w, uint64_t key0, uint64_t key1, uint64_t step,
                          double delta, int32_t *n_acc, int n_tau, double *tau) {
    int nb = (c->m + n_tau + 63) / 64;
    advance_kernel<<<nb, 64, 0, c->stream>>>(walkers, w, c->m, c->nuc, c->gpar, c->n_nuc, c->Ng, key0, key1, step, delta,
                                             n_acc, n_tau, c->lambda, tau);
    return hipGetLastError();
}

hipError_t launch_sample_tau(const mcmp2_ctx *c, uint64_t key0, uint64_t key1, uint64_t step, int n_tau,
                             double *tau) {
    sample_tau_kernel<<<(n_tau + 63) / 64, 64, 0, c->stream>>>(key0, key1, step, n_tau, c->lambda, tau);
    return hipGetLastError();
}
