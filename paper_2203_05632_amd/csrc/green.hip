// Green's functions and pair contraction of the MC-MP2 integrand (Sec. III
// of the paper, the G+ / G- definitions and Eq. redundant), FP64 and FP32
// operands (FP64 contraction in both).
//
// For tau sample t the operands are the spinor values psi[k][r] scaled by
//   s_k = exp(+eps_k tau)  (occupied, G-)   or   exp(-eps_k tau)  (virtual, G+),
// and the Green's functions over all 8m x 8m rows are
//   G(x, y) = sum_k s_k psi[k][x] conj(psi[k][y]).
// Only the 8x8 blocks of walker pairs p < q enter the estimator, and
// G(y, x) = G(x, y)^dagger, so the kernel walks the upper triangle of
// 32x32-row block tiles (4 walker pairs per side).  A workgroup owns one block
// tile and computes G- and G+ for up to two tau samples from a single pass
// over the operands, on FP64 MFMA with complex numbers as real pairs.  With
// psi_x = a + ib and psi_y = c + id the entry is Re G = sum a c + b d,
// Im G = sum b c - a d; the kernel forms it from three real products instead
// of four (the 3M / Gauss form of complex multiplication):
//   T1 = sum a c,  T2 = sum b d,  T3 = sum (a + b)(c - d),
//   Re G = T1 + T2,  Im G = T3 - T1 + T2,
// which cuts the MFMA work by a quarter; the rounding error of Im G stays of
// the order of the unit roundoff times |a||c| + |b||d| summed over k.
// The tile never leaves the chip: per tau each wave stages its 16x16 G- and
// G+ sub-tiles in LDS and contracts the (up to) four walker pairs they cover,
//   D = Tr[G-(3,1) G+(1,3)] Tr[G-(4,2) G+(2,4)],
//   X = Tr[G-(3,1) G+(1,4) G-(4,2) G+(2,3)],
// (1 = r1p, 2 = r2p, 3 = r1q, 4 = r2q; G(3,1) = G(1,3)^dagger), and weights
// each pair by N_g^2 / (g(1) g(2) g(3) g(4) w(tau)) -- the 1/(r12 r34) of the
// integrand cancels the 1/r of the two pair weights.  Per wave it writes the
// direct part -Re(D)/2 and the exchange part +Re(X)/2 summed over its pairs;
// a second kernel reduces them with compensated (Neumaier) summation in a
// fixed order, so results are bitwise reproducible.  (Folding that reduction
// into the last block to finish was measured slower: the device-scope release
// fence it needs writes back each XCD's L2 once per block.)
//
// Work order: workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2.  The host builds the wave-slot list so that the tile pairs
// an XCD receives come from compact bands of tile rows and columns whose psi
// slices fit that XCD's L2 (build_green_work).
#include <algorithm>

#include <type_traits>

#include "contract.hpp"

namespace {

// Neumaier (improved Kahan) summation: s + c carries the running total.
__device__ inline void neumaier_add(double &s, double &c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// Compensated sum over the n_slots partials of tau t by one block of 256
// threads: per-thread sums over a fixed stride, then a fixed-shape tree
// (wave shuffles, then the 4 wave totals in order) -- the same order in every
// launch runs it, so the result is bitwise reproducible.  A thread's terms
// are fetched RB at a time before they are added, so their loads overlap
// instead of each waiting for the previous add; a term past the end reads as
// 0.0, which leaves the sum and its compensation unchanged.
__device__ inline void reduce_tau(const double *__restrict__ partial, int n_slots, int t, double inv_pairs,
                                  double *__restrict__ e2_out, double (*sh)[4]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int RB = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const d2 *src = reinterpret_cast<const d2 *>(partial) + (size_t)t * n_slots;
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    for (int i0 = threadIdx.x; i0 < n_slots; i0 += 256 * RB) {
        d2 v[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int i = i0 + 256 * u;
            v[u] = i < n_slots ? src[i] : d2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            neumaier_add(s0, c0, v[u].x);
            neumaier_add(s1, c1, v[u].y);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double s0o = __shfl_down(s0, off, 64), c0o = __shfl_down(c0, off, 64);
        const double s1o = __shfl_down(s1, off, 64), c1o = __shfl_down(c1, off, 64);
        if (lane < off) {
            neumaier_add(s0, c0, s0o);
            c0 += c0o;
            neumaier_add(s1, c1, s1o);
            c1 += c1o;
        }
    }
    if (lane == 0) {
        sh[wave][0] = s0;
        sh[wave][1] = c0;
        sh[wave][2] = s1;
        sh[wave][3] = c1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = sh[0][0], b0 = sh[0][1], a1 = sh[0][2], b1 = sh[0][3];
        for (int w = 1; w < 4; ++w) {
            neumaier_add(a0, b0, sh[w][0]);
            b0 += sh[w][1];
            neumaier_add(a1, b1, sh[w][2]);
            b1 += sh[w][3];
        }
        const double d = (a0 + b0) * inv_pairs, x = (a1 + b1) * inv_pairs;
        e2_out[3 * t] = d;
        e2_out[3 * t + 1] = x;
        e2_out[3 * t + 2] = d + x;
    }
    __syncthreads();
}

// Block tile: 32 x 32 rows (4 walker pairs x 4 walker pairs), one 16 x 16
// sub-tile per wave (wave w: rows 16 (w >> 1), cols 16 (w & 1)).  The K
// dimension (spinors) is streamed in chunks of KC through double-buffered
// LDS panels shared by the 4 waves: A = the 32 rows of the P range, B = the
// 32 rows of the Q range, both [k][row] with the row fastest.
constexpr int KC = 16;

// Operand type of the Green's GEMM: FP64 (FP64 mode) or FP32 (FP32 mode; psi
// from the FP32 spinor GEMM, FP32 MFMA accumulation, the contraction in FP64
// as in FP64 mode).  FP64 uses the 3M form (T1, T2, T3); FP32 keeps the four
// real products (re and im accumulators in T1, T2): its error budget against
// the FP64 result is set by FP32 rounding and 3M would loosen it.
template <typename T>
struct GOp;
template <>
struct GOp<double> {
    using V2 = double2;
    using Acc = d4v;
    static constexpr bool M3 = true;
    __device__ static Acc mfma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int v, int lk) { return 4 * v + lk; }  // MFMA f64 result row of element v
};
template <>
struct GOp<float> {
    using V2 = float2;
    typedef float Acc __attribute__((ext_vector_type(4)));
    static constexpr bool M3 = false;
    __device__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int v, int lk) { return 4 * lk + v; }  // MFMA f32 result row of element v
};

// One K-step of 4 spinors (x = P-range operand, scaled per tau; y = Q-range
// operand).  FP64: the three real products of the 3M form into t1, t2, t3;
// FP32: Re G into t1 (a c + b d), Im G into t2 (b c - a d).
template <typename T, int NT>
__device__ inline void mfma_kstep(const typename GOp<T>::V2 *__restrict__ pa, const typename GOp<T>::V2 *__restrict__ pb,
                                  const double (&s)[NT], typename GOp<T>::Acc (&t1)[NT],
                                  typename GOp<T>::Acc (&t2)[NT], typename GOp<T>::Acc (&t3)[NT]) {
    using O = GOp<T>;
    const typename O::V2 x = *pa, y = *pb;
    T a[NT], b[NT];
    for (int t = 0; t < NT; ++t) {
        a[t] = x.x * (T)s[t];
        b[t] = x.y * (T)s[t];
    }
    if constexpr (O::M3) {
        const T xs = x.x + x.y, yd = y.x - y.y;
        T ab[NT];
        for (int t = 0; t < NT; ++t) ab[t] = xs * (T)s[t];
        for (int t = 0; t < NT; ++t) t1[t] = O::mfma(a[t], y.x, t1[t]);
        for (int t = 0; t < NT; ++t) t2[t] = O::mfma(b[t], y.y, t2[t]);
        for (int t = 0; t < NT; ++t) t3[t] = O::mfma(ab[t], yd, t3[t]);
    } else {
        for (int t = 0; t < NT; ++t) t1[t] = O::mfma(a[t], y.x, t1[t]);
        for (int t = 0; t < NT; ++t) t2[t] = O::mfma(b[t], y.x, t2[t]);
        for (int t = 0; t < NT; ++t) t1[t] = O::mfma(b[t], y.y, t1[t]);
        for (int t = 0; t < NT; ++t) t2[t] = O::mfma(-a[t], y.y, t2[t]);
    }
}

template <typename V2>
__device__ inline void chunk_load(const V2 *__restrict__ psi, int R, int rp, int rq, int kc, int k_hi, int e0, int e1,
                                  V2 &ra0, V2 &ra1, V2 &rb0, V2 &rb1) {
    const int k0 = kc + (e0 >> 5), k1 = kc + (e1 >> 5);
    const size_t o0 = (size_t)k0 * R + (e0 & 31), o1 = (size_t)k1 * R + (e1 & 31);
    const V2 z = {0, 0};
    ra0 = k0 < k_hi ? psi[o0 + rp] : z;
    rb0 = k0 < k_hi ? psi[o0 + rq] : z;
    ra1 = k1 < k_hi ? psi[o1 + rp] : z;
    rb1 = k1 < k_hi ? psi[o1 + rq] : z;
}

template <typename V2>
__device__ inline void chunk_store(V2 (*buf)[KC][32], int e0, int e1, const V2 &ra0, const V2 &ra1, const V2 &rb0,
                                   const V2 &rb1) {
    buf[0][e0 >> 5][e0 & 31] = ra0;
    buf[1][e0 >> 5][e0 & 31] = rb0;
    buf[0][e1 >> 5][e1 & 31] = ra1;
    buf[1][e1 >> 5][e1 & 31] = rb1;
}

// tau scalings of one chunk: thread tid < 4 KC loads s_t[k] for t = tid / KC, k = kc + tid % KC
__device__ inline double scale_load(const double *__restrict__ sc, int nsp, int nt, int kc, int k_hi, int tid) {
    const int t = tid / KC, k = kc + tid % KC;
    return (t < nt && k < k_hi) ? sc[(size_t)t * nsp + k] : 0.0;
}

// Stream spinors k in [k_lo, k_hi) through the LDS panels in chunks of KC
// (the next chunk's global loads are in flight while the current one feeds
// the MFMAs) and accumulate this wave's sub-tile for NT tau samples.
// TWO: two register stages of prefetch (used by the gradient kernels, which
// run at two waves per SIMD with or without the second stage; the forward
// kernels would lose a wave per SIMD to its registers).
template <typename T, int NT, bool TWO>
__device__ inline void stream_k(const typename GOp<T>::V2 *__restrict__ psi, const double *__restrict__ sc, int nsp,
                                int R, int rp, int rq, int k_lo, int k_hi, typename GOp<T>::V2 (*panel)[2][KC][32],
                                double (*spanel)[4 * KC], typename GOp<T>::Acc (&t1)[NT],
                                typename GOp<T>::Acc (&t2)[NT], typename GOp<T>::Acc (&t3)[NT]) {
    using V2 = typename GOp<T>::V2;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wp = wave >> 1, wq = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    // Cooperative load of one chunk: thread element e in {tid, tid + 256} is
    // (k = kc + e / 32, row = e % 32) of both panels; k >= k_hi reads as zero.
    // (Plain scalars here: a lambda version over register arrays crashes the
    // ROCm 7.2 AMDGPU backend in machine copy propagation.)
    const int e0 = tid, e1 = tid + 256;
    const int n_chunks = (k_hi - k_lo + KC - 1) / KC;
#define GK_COMPUTE(BUF)                                                                                             \
    _Pragma("unroll") for (int ks = 0; ks < KC; ks += 4) {                                                          \
        double s[NT];                                                                                               \
        for (int t = 0; t < NT; ++t) s[t] = spanel[BUF][t * KC + ks + lk];                                          \
        mfma_kstep<T, NT>(&panel[BUF][0][ks + lk][16 * wp + li], &panel[BUF][1][ks + lk][16 * wq + li], s, t1, t2, t3); \
    }
    if constexpr (TWO) {
        // Two register stages: the loads of chunk c + 2 are issued before chunk
        // c is multiplied and go to LDS after chunk c + 1 is; past the last
        // chunk the loads re-read it (branch-free, so the compiler's waits at
        // each LDS store cover only the older stage).
        V2 ra0, ra1, rb0, rb1, qa0, qa1, qb0, qb1;
        double sv, sw;
        const int k_last = k_lo + (n_chunks - 1) * KC;
        chunk_load(psi, R, rp, rq, k_lo, k_hi, e0, e1, ra0, ra1, rb0, rb1);
        sv = scale_load(sc, nsp, NT, k_lo, k_hi, tid);
        chunk_load(psi, R, rp, rq, min(k_lo + KC, k_last), k_hi, e0, e1, qa0, qa1, qb0, qb1);
        sw = scale_load(sc, nsp, NT, min(k_lo + KC, k_last), k_hi, tid);
        chunk_store(panel[0], e0, e1, ra0, ra1, rb0, rb1);
        if (tid < 4 * KC) spanel[0][tid] = sv;
        __syncthreads();
        for (int c = 0; c < n_chunks; c += 2) {
            const int k2 = min(k_lo + (c + 2) * KC, k_last), k3 = min(k_lo + (c + 3) * KC, k_last);
            chunk_load(psi, R, rp, rq, k2, k_hi, e0, e1, ra0, ra1, rb0, rb1);  // (q) holds chunk c + 1
            sv = scale_load(sc, nsp, NT, k2, k_hi, tid);
            GK_COMPUTE(0)
            if (c + 1 < n_chunks) {
                chunk_store(panel[1], e0, e1, qa0, qa1, qb0, qb1);
                if (tid < 4 * KC) spanel[1][tid] = sw;
            }
            __syncthreads();
            if (c + 1 >= n_chunks) break;
            chunk_load(psi, R, rp, rq, k3, k_hi, e0, e1, qa0, qa1, qb0, qb1);  // (r) holds chunk c + 2
            sw = scale_load(sc, nsp, NT, k3, k_hi, tid);
            GK_COMPUTE(1)
            if (c + 2 < n_chunks) {
                chunk_store(panel[0], e0, e1, ra0, ra1, rb0, rb1);
                if (tid < 4 * KC) spanel[0][tid] = sv;
            }
            __syncthreads();
        }
    } else {
        V2 ra0, ra1, rb0, rb1;
        double sv;
        chunk_load(psi, R, rp, rq, k_lo, k_hi, e0, e1, ra0, ra1, rb0, rb1);
        sv = scale_load(sc, nsp, NT, k_lo, k_hi, tid);
        chunk_store(panel[0], e0, e1, ra0, ra1, rb0, rb1);
        if (tid < 4 * KC) spanel[0][tid] = sv;
        __syncthreads();
        for (int c = 0; c < n_chunks; ++c) {
            const int buf = c & 1;
            const int kc = k_lo + c * KC;
            if (c + 1 < n_chunks) {
                chunk_load(psi, R, rp, rq, kc + KC, k_hi, e0, e1, ra0, ra1, rb0, rb1);
                sv = scale_load(sc, nsp, NT, kc + KC, k_hi, tid);
            }
            // operands of this chunk come from LDS only, so the next chunk's
            // global loads stay in flight across all of its MFMAs
            GK_COMPUTE(buf)
            if (c + 1 < n_chunks) {
                chunk_store(panel[buf ^ 1], e0, e1, ra0, ra1, rb0, rb1);
                if (tid < 4 * KC) spanel[buf ^ 1][tid] = sv;
            }
            __syncthreads();
        }
    }
#undef GK_COMPUTE
}

// G entry v of a lane's accumulators from the GEMM's partial sums
template <typename T>
__device__ inline cplx g_entry(const typename GOp<T>::Acc &t1, const typename GOp<T>::Acc &t2,
                               const typename GOp<T>::Acc &t3, int v) {
    if constexpr (GOp<T>::M3)
        return {t1[v] + t2[v], (t3[v] - t1[v]) + t2[v]};
    else
        return {(double)t1[v], (double)t2[v]};
}

// grid: (n_slots / 4, tau chunks); block (x, y) takes work item x and tau
// samples t0 .. t0 + NT - 1, t0 = y NT.  T: operand type (double / float).
// GRAD: also write, per walker pair, the 8x8 blocks of the Hermitian adjoint
// matrices H- and H+ (gradient of the step value with respect to the entries
// of G- and G+, folded as Gbar + Gbar^H) into Hm / Hp [n_tau][R][R] complex.
// BREIT: Gaunt / Breit interaction in the contraction (rhat [m_pad][4] unit
// vectors of r1p - r2p, gauge = weight of the second Breit term; one tau per
// block).  With GRAD and BREIT the kernel copies, for every pair p < q < m,
// G-(1,3), G-(2,4) and the four 4x4 blocks of G+ into the pair's blocks of
// Hm / Hp instead, for breit_adjoint_kernel.
template <typename T, int NT, bool GRAD, bool BREIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT == 1 && !GRAD && !BREIT ? 4 : 2))) void
green_contract_kernel(const void *__restrict__ psi_, const double *__restrict__ scale,
                      const double *__restrict__ wtau, const double *__restrict__ hinv, const int *__restrict__ tiles,
                      const int *__restrict__ work, int n_slots, int R, int no, int nsp, int m,
                      double *__restrict__ partial, double2 *__restrict__ Hm, double2 *__restrict__ Hp, double cgrad,
                      const double *__restrict__ rhat, double gauge) {
    using O = GOp<T>;
    using V2 = typename O::V2;
    using Acc = typename O::Acc;
    const int t0 = (int)blockIdx.y * NT;
    // 2 buffers x (A, B) x KC x 32 complex operands (32 KB FP64, 16 KB FP32),
    // reused for the FP64 G tiles of the epilogue (4 waves x 512 complex = 32 KB)
    constexpr int PANEL_BYTES = 2 * 2 * KC * 32 * (int)sizeof(V2);
    constexpr int EPI_BYTES = 4 * 512 * (int)sizeof(cplx);
    __shared__ __align__(16) unsigned char smem[PANEL_BYTES > EPI_BYTES ? PANEL_BYTES : EPI_BYTES];
    __shared__ double spanel[2][4 * KC];  // tau scalings of the buffered chunks
    V2(*panel)[2][KC][32] = reinterpret_cast<V2(*)[2][KC][32]>(smem);
    const V2 *psi = reinterpret_cast<const V2 *>(psi_);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int item = work[blockIdx.x];
    if (item < 0) {  // padding block: zero partials
        for (int t = 0; t < NT; ++t)
            if (lane == 0) {
                double *out = partial + ((size_t)(t0 + t) * n_slots + 4 * blockIdx.x + wave) * 2;
                out[0] = out[1] = 0.0;
            }
        return;
    }
    const int PT = tiles[2 * item], QT = tiles[2 * item + 1];
    const int rp = 32 * PT, rq = 32 * QT;
    const double *sc = scale + (size_t)t0 * nsp;

    // occupied spinors -> G-, then virtual spinors -> G+; G- is assembled
    // (FP64) before the G+ pass to free its partial sums' registers
    cplx gm[NT][4];
    {
        Acc m1[NT], m2[NT], m3[NT];
        for (int t = 0; t < NT; ++t) m1[t] = m2[t] = m3[t] = Acc{0, 0, 0, 0};
        stream_k<T, NT, GRAD && !BREIT>(psi, sc, nsp, R, rp, rq, 0, no, panel, spanel, m1, m2, m3);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) gm[t][v] = g_entry<T>(m1[t], m2[t], m3[t], v);
    }
    Acc p1[NT], p2[NT], p3[NT];
    for (int t = 0; t < NT; ++t) p1[t] = p2[t] = p3[t] = Acc{0, 0, 0, 0};
    stream_k<T, NT, GRAD && !BREIT>(psi, sc, nsp, R, rp, rq, no, nsp, panel, spanel, p1, p2, p3);

    // epilogue: per tau, stage the wave's G- and G+ sub-tiles in LDS and contract
    cplx *Gm = reinterpret_cast<cplx *>(smem) + wave * 512;
    cplx *Gp = Gm + 256;
    const int slot = 4 * blockIdx.x + wave;
#pragma unroll  // constant indices keep the accumulators in registers
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = O::row(v, lk);
            const cplx gp = g_entry<T>(p1[t], p2[t], p3[t], v);
            Gm[i * 16 + li] = gm[t][v];
            Gp[i * 16 + li] = gp;
            if constexpr (GRAD && BREIT) {
                const int row = rp + 16 * (wave >> 1) + i, col = rq + 16 * (wave & 1) + li;
                if ((row >> 3) < (col >> 3) && (col >> 3) < m) {
                    // G- only in its (1,3) and (2,4) blocks: the adjoint reads and
                    // overwrites those, and H-(1,4), H-(2,3) stay zero
                    const size_t o = (size_t)(t0 + t) * R * R + (size_t)row * R + col;
                    if (((row ^ col) & 4) == 0) Hm[o] = double2{gm[t][v].re, gm[t][v].im};
                    Hp[o] = double2{gp.re, gp.im};
                }
            }
        }
        // The staged sub-tiles are private to the wave (the K loop ended with a
        // block barrier) and one wave's LDS accesses complete in order, so a
        // wave barrier orders the staging against the contraction's reads.
        __builtin_amdgcn_wave_barrier();
        if constexpr (BREIT)
            contract_pairs_breit(Gm, Gp, PT, QT, m, hinv, rhat, gauge, wtau[t0 + t],
                                 partial + ((size_t)(t0 + t) * n_slots + slot) * 2);
        else
            contract_pairs<GRAD, double2>(Gm, Gp, PT, QT, m, hinv, wtau[t0 + t], cgrad, R,
                                          partial + ((size_t)(t0 + t) * n_slots + slot) * 2,
                                          GRAD ? Hm + (size_t)(t0 + t) * R * R : nullptr,
                                          GRAD ? Hp + (size_t)(t0 + t) * R * R : nullptr);
        __builtin_amdgcn_wave_barrier();  // the sub-tiles are rewritten for the next tau
    }
}

// Adjoint of the Gaunt / Breit contraction.  Grid as green_contract_kernel's
// with one tau per block row (x: work-list entry, y: tau); wave (wp, wq) takes
// the same 16x16 sub-tiles and walker pairs.  On entry Hm / Hp [n_tau][R][R]
// hold, in the 8x8 blocks of the pairs p < q < m, G-(1,3), G-(2,4) (H-(1,4)
// and H-(2,3) are zero, as everywhere) and all of G+ (written by the Green's
// kernel); each pair reads its own blocks and overwrites those with its
// adjoint blocks, writing their Hermitian partners into the (q, p) blocks,
// which no pair reads.  Diagonal and padding blocks are never written.
// HT: double2 (FP64, FP32 modes) or uint32_t (BF16 pairs: BF16 / FP16 modes,
// G read as BF16 pairs, the adjoint formed in FP64 and rounded once).
template <typename HT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void
breit_adjoint_kernel(HT *__restrict__ Hm, HT *__restrict__ Hp, const double *__restrict__ wtau,
                     const double *__restrict__ hinv, const int *__restrict__ tiles, const int *__restrict__ work,
                     int R, int m, double cgrad, const double *__restrict__ rhat, double gauge) {
    __shared__ __align__(16) cplx sg[4][2][256];
    const int item = work[blockIdx.x];
    if (item < 0) return;
    const int t = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wp = wave >> 1, wq = wave & 1;
    const int PT = tiles[2 * item], QT = tiles[2 * item + 1];
    const int p0 = kTileWalkers * PT + 2 * wp, q0 = kTileWalkers * QT + 2 * wq;
    if (p0 >= q0 + 1 || q0 >= m) return;  // no pair p < q < m in this wave's sub-tile
    HT *hm = Hm + (size_t)t * R * R, *hp = Hp + (size_t)t * R * R;
    cplx *Gm = sg[wave][0], *Gp = sg[wave][1];
    const int li = lane & 15, lk = lane >> 4;
    const size_t r0 = 8 * (size_t)p0, c0 = 8 * (size_t)q0;
    auto wide = [](HT x) {
        if constexpr (std::is_same_v<HT, uint32_t>)  // BF16 pair, real part low
            return cplx{(double)__uint_as_float(x << 16), (double)__uint_as_float(x & 0xffff0000u)};
        else
            return cplx{x.x, x.y};
    };
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + lk;
        const size_t o = (r0 + i) * R + c0 + li;
        const HT x = hm[o], y = hp[o];
        Gm[i * 16 + li] = wide(x);
        Gp[i * 16 + li] = wide(y);
    }
    // the sub-tiles are private to the wave, whose LDS accesses complete in order
    __builtin_amdgcn_wave_barrier();
    const int pi = lane >> 4, pp = pi >> 1, qq = pi & 1;
    const int p = p0 + pp, q = q0 + qq;
    breit_adjoint_pair(Gm + 8 * pp * 16 + 8 * qq, Gp + 8 * pp * 16 + 8 * qq, 16, p, q, p < q && q < m, hinv, rhat,
                       gauge, wtau[t], cgrad, R, hm, hp);
}

// One block per tau sample.
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial, int n_slots, double inv_pairs,
                                                     double *__restrict__ e2_out) {
    __shared__ double sh[4][4];
    reduce_tau(partial, n_slots, blockIdx.x, inv_pairs, e2_out, sh);
}

// The step value V = (1/n_tau) sum_t e2_out[t][2] (the tau average of
// Eq. redundant's pair averages), summed in tau order with compensation.
__global__ __launch_bounds__(64) void step_value_kernel(const double *__restrict__ e2_out, int n_tau,
                                                        double *__restrict__ value) {
    if (threadIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int t = 0; t < n_tau; ++t) neumaier_add(s, c, e2_out[3 * t + 2]);
    value[0] = (s + c) / (double)n_tau;
}

}  // namespace

// Tile pairs (P <= Q) of T block tiles are grouped into super-blocks of bands
// of B tiles (I <= J) so that the psi rows of two bands (2 B tiles) fit in
// ~2.5 MB of an XCD's 4 MB L2.  Super-blocks go to the 8 XCD lists largest
// first to the least loaded list; the lists are padded to equal length (-1)
// and interleaved so that workgroup b (dispatched to XCD b mod 8) takes entry
// b / 8 of list b mod 8.  Every XCD then works through its own list: B is the
// widest band within the L2 budget whose longest list is at most 20% above
// the mean.  (At 128 walker pairs the L2 budget alone allows 14-tile bands
// for FP32 rows and 27-tile bands for BF16 rows: 6 and 3 super-blocks, two and
// five XCDs idle.  A 3% bound, i.e. narrower bands, measured no faster and
// doubled the FP64 kernel's HBM reads.)
void build_green_work(int T, double tile_bytes, std::vector<int> &work) {
    constexpr int kXcd = 8;
    auto tp_index = [T](int P, int Q) { return P * T - P * (P - 1) / 2 + (Q - P); };
    auto deal = [&](int B, std::vector<std::vector<int>> &lists) {
        const int nbands = (T + B - 1) / B;
        std::vector<std::vector<int>> blocks;
        for (int I = 0; I < nbands; ++I)
            for (int J = I; J < nbands; ++J) {
                std::vector<int> items;
                for (int P = I * B; P < std::min(T, (I + 1) * B); ++P)
                    for (int Q = std::max(P, J * B); Q < std::min(T, (J + 1) * B); ++Q)
                        items.push_back(tp_index(P, Q));
                if (!items.empty()) blocks.push_back(std::move(items));
            }
        std::stable_sort(blocks.begin(), blocks.end(),
                         [](const std::vector<int> &x, const std::vector<int> &y) { return x.size() > y.size(); });
        lists.assign(kXcd, {});
        for (auto &blk : blocks) {
            size_t best = 0;
            for (size_t x = 1; x < lists.size(); ++x)
                if (lists[x].size() < lists[best].size()) best = x;
            lists[best].insert(lists[best].end(), blk.begin(), blk.end());
        }
        size_t len = 0;
        for (auto &l : lists) len = std::max(len, l.size());
        return len;
    };
    const int b_l2 = std::min(T, std::max(1, (int)(2.5e6 / (2.0 * tile_bytes))));
    const double mean = (double)T * (T + 1) / 2 / kXcd;
    std::vector<std::vector<int>> lists;
    int B = b_l2;
    for (; B > 1; --B)
        if (deal(B, lists) <= 1.2 * mean) break;
    const size_t len = deal(B, lists);
    work.assign(kXcd * len, -1);
    for (size_t b = 0; b < work.size(); ++b) {
        const auto &l = lists[b % kXcd];
        if (b / kXcd < l.size()) work[b] = l[b / kXcd];
    }
}

// Tau samples per block: NT divides n_tau (every block of the launch has NT
// samples), and the launch's makespan is modelled as (blocks per CU, rounded
// up) x NT.  Larger NT shares each operand panel across more samples, so the
// largest NT within 5% of the best makespan is taken.  NT is at most 2: with
// three accumulator tiles per sample and function, NT = 4 leaves one wave per
// SIMD and was measured slower than NT = 2 on the 512-pair workload.
constexpr int kMaxTauChunk = 2;

int green_tau_chunk(int nblocks, int n_tau, int n_cu) {
    auto cost = [&](int nt) { return (double)((nblocks * (n_tau / nt) + n_cu - 1) / n_cu) * nt; };
    double best = 1e300;
    for (int nt = 1; nt <= kMaxTauChunk; ++nt)
        if (n_tau % nt == 0) best = std::min(best, cost(nt));
    for (int nt = kMaxTauChunk; nt >= 1; --nt)
        if (n_tau % nt == 0 && cost(nt) <= 1.05 * best) return nt;
    return 1;
}

namespace {

// One launch of NTV tau samples per block: the gradient variant, the Gaunt /
// Breit variant (one tau per block only) or the plain estimator.
template <typename T, int NTV>
void launch_green_dispatch(const mcmp2_ctx *c, dim3 grid, bool grad, bool breit, double cgrad) {
    double2 *Hm = reinterpret_cast<double2 *>(c->Hm), *Hp = reinterpret_cast<double2 *>(c->Hp);
    if constexpr (NTV == 1) {
        if (grad && breit) {  // G blocks to Hm / Hp, then their adjoint in place
            const double gauge = c->interaction == MCMP2_BREIT ? 1.0 : 0.0;
            green_contract_kernel<T, 1, true, true><<<grid, 256, 0, c->stream>>>(
                c->psi, c->scale, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->no, c->nsp, c->m,
                c->partial, Hm, Hp, cgrad, c->rhat, gauge);
            breit_adjoint_kernel<double2><<<grid, 256, 0, c->stream>>>(Hm, Hp, c->wtau, c->hinv, c->tiles, c->work,
                                                                        c->R, c->m, cgrad, c->rhat, gauge);
            return;
        }
    }
    if (grad) {
        green_contract_kernel<T, NTV, true, false><<<grid, 256, 0, c->stream>>>(
            c->psi, c->scale, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->no, c->nsp, c->m,
            c->partial, Hm, Hp, cgrad, c->rhat, 0.0);
        return;
    }
    if constexpr (NTV == 1) {
        if (breit) {
            const double gauge = c->interaction == MCMP2_BREIT ? 1.0 : 0.0;
            green_contract_kernel<T, 1, false, true><<<grid, 256, 0, c->stream>>>(
                c->psi, c->scale, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->no, c->nsp, c->m,
                c->partial, nullptr, nullptr, 0.0, c->rhat, gauge);
            return;
        }
    }
    green_contract_kernel<T, NTV, false, false><<<grid, 256, 0, c->stream>>>(
        c->psi, c->scale, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->no, c->nsp, c->m, c->partial,
        nullptr, nullptr, 0.0, c->rhat, 0.0);
}

template <typename T, int NTV>
void launch_green_nt(const mcmp2_ctx *c, dim3 grid, bool grad, bool breit, double cgrad) {
    const int ps = prof_begin(c, MCMP2_K_GREEN_GEMM);
    launch_green_dispatch<T, NTV>(c, grid, grad, breit, cgrad);
    (void)prof_end(c, ps, MCMP2_K_GREEN_GEMM);
}

template <typename T>
void launch_green_typed(const mcmp2_ctx *c, dim3 grid, int nt, bool grad, bool breit, double cgrad) {
    if (nt == 1)
        launch_green_nt<T, 1>(c, grid, grad, breit, cgrad);
    else
        launch_green_nt<T, 2>(c, grid, grad, breit, cgrad);
}

}  // namespace

// FP64 and FP32 modes (the operand type follows the context's precision).
hipError_t launch_green_contract(const mcmp2_ctx *c, int n_tau, bool grad) {
    // gradient of the step value (mean over tau of the pair average): c = -1/2 / (mC2 n_tau)
    const double cgrad = -0.5 / (0.5 * (double)c->m * (double)(c->m - 1) * (double)n_tau);
    const int nblocks = c->n_slots / 4;  // one work-list entry per block, four partial slots
    const bool breit = c->interaction != MCMP2_COULOMB;
    // one tau per block with the Gaunt / Breit contraction: its epilogue
    // needs the registers that a second tau's accumulators would hold
    const int nt = breit ? 1 : green_tau_chunk(nblocks, n_tau, c->n_cu);
    const dim3 grid(nblocks, n_tau / nt);
    if (c->precision == MCMP2_FP32)
        launch_green_typed<float>(c, grid, nt, grad, breit, cgrad);
    else
        launch_green_typed<double>(c, grid, nt, grad, breit, cgrad);
    return hipGetLastError();
}


// BF16 / FP16 modes: the Gaunt / Breit adjoint on the G blocks the 32 x 32-tile
// Green's kernel left in Hm / Hp (BF16 pairs), grid as that kernel's.
hipError_t launch_breit_adjoint_lp(const mcmp2_ctx *c, int n_tau, double cgrad) {
    const double gauge = c->interaction == MCMP2_BREIT ? 1.0 : 0.0;
    breit_adjoint_kernel<uint32_t><<<dim3(c->n_slots / 4, n_tau), 256, 0, c->stream>>>(
        reinterpret_cast<uint32_t *>(c->Hm), reinterpret_cast<uint32_t *>(c->Hp), c->wtau, c->hinv, c->tiles, c->work,
        c->R, c->m, cgrad, c->rhat, gauge);
    return hipGetLastError();
}

hipError_t launch_reduce(const mcmp2_ctx *c, int n_tau, double *e2_out) {
    const double inv_pairs = 1.0 / (0.5 * (double)c->m * (double)(c->m - 1));
    const int n_slots = green_big_selected(c, n_tau) ? 8 * c->n_tp16 : c->n_slots;
    reduce_kernel<<<n_tau, 256, 0, c->stream>>>(c->partial, n_slots, inv_pairs, e2_out);
    return hipGetLastError();
}

hipError_t launch_step_value(const mcmp2_ctx *c, const double *e2_out, int n_tau, double *value) {
    step_value_kernel<<<1, 64, 0, c->stream>>>(e2_out, n_tau, value);
    return hipGetLastError();
}
