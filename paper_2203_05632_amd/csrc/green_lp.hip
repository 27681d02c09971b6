// Low-precision Green's functions (FP32, BF16, FP16 operands on MFMA with
// FP32 accumulation) followed by the same FP64 pair contraction as the FP64
// path (Sec. III of the paper: G+ / G- and the redundant-walker estimator).
//
// Operands.  For tau sample t, lp_operands writes
//   U_t[row][K] = psi[k][row] * sqrt(s_t[k]),  K = 2 k (+1 for the imaginary part),
// with s_t[k] = exp(+eps_k tau) (occupied) / exp(-eps_k tau) (virtual)
// computed and square-rooted in FP64, the product rounded once to the
// operand type.  The symmetric square-root scaling keeps both operands within
// the same range (FP16 included; terms below FP16's range flush to zero and
// are weighted by exp(-eps tau) < 2^-24 relative to the largest).  Occupied
// spinors fill K in [0, Ko), virtual ones [Ko, Ko + Kv), each padded with
// zeros to a multiple of the K chunk.
//
// With complex numbers interleaved along K, G(x, y) = sum_k s_k psi_x conj(psi_y)
// is two real GEMMs over the same A rows:
//   Re G = U_x . U_y,   Im G = U_x . W_y,  W = (-im, re) pairs of U_y,
// W being formed from the B operand in registers.
#include <algorithm>

#include "contract.hpp"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

// Reals of K per LDS chunk (FP32: 32 = one pass of 8 K-steps over 4 lane
// groups; BF16/FP16: 64 = two 16x16x32 K-steps) and the padded LDS row
// length: 16 extra bytes per row so that the 16-byte reads of 8 consecutive
// rows fall in distinct banks.
template <typename T>
constexpr int lkc() {
    return sizeof(T) == 4 ? 32 : 64;
}
template <typename T>
constexpr int lrow() {
    return lkc<T>() + 16 / (int)sizeof(T);
}

template <typename T>
__device__ inline T to_op(double v);
template <>
__device__ inline float to_op<float>(double v) {
    return (float)v;
}
template <>
__device__ inline __bf16 to_op<__bf16>(double v) {
    return (__bf16)v;
}
template <>
__device__ inline _Float16 to_op<_Float16>(double v) {
    return (_Float16)v;
}

// grid (R / 64, ceil(nsp / 32), n_tau); psi float2 [nsp][R] -> U_t [R][Ktot]
template <typename T>
__global__ __launch_bounds__(256) void lp_operands_kernel(const float2 *__restrict__ psi,
                                                          const double *__restrict__ scale, int R, int nsp, int no,
                                                          int Ko, int Ktot, T *__restrict__ U) {
    __shared__ float2 tile[32][65];
    __shared__ double sq[32];
    const int r0 = 64 * blockIdx.x, k0 = 32 * blockIdx.y, t = blockIdx.z;
    const int tid = threadIdx.x;
    if (tid < 32) {
        const int k = k0 + tid;
        sq[tid] = k < nsp ? sqrt(scale[(size_t)t * nsp + k]) : 0.0;
    }
    for (int e = tid; e < 32 * 64; e += 256) {  // coalesced along rows
        const int kk = e >> 6, r = e & 63, k = k0 + kk;
        tile[kk][r] = k < nsp ? psi[(size_t)k * R + r0 + r] : float2{0.f, 0.f};
    }
    __syncthreads();
    T *Ut = U + (size_t)t * R * Ktot;
    for (int e = tid; e < 32 * 64; e += 256) {  // coalesced along K within a row
        const int r = e >> 5, kk = e & 31, k = k0 + kk;
        if (k >= nsp) continue;
        const int K = k < no ? 2 * k : Ko + 2 * (k - no);
        const float2 v = tile[kk][r];
        T *o = Ut + (size_t)(r0 + r) * Ktot + K;
        o[0] = to_op<T>((double)v.x * sq[kk]);
        o[1] = to_op<T>((double)v.y * sq[kk]);
    }
}

// MFMA wrappers: 16x16 output tiles, result D[4 (l / 16) + v][l % 16] in element v.
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {  // v_mfma_f32_16x16x4f32: lane holds A[l%16][l/16], B[l/16][l%16]
    static constexpr int K = 4;
};
template <>
struct Mfma<__bf16> {  // v_mfma_f32_16x16x32_bf16: lane holds A[l%16][8(l/16)+j], B[8(l/16)+j][l%16]
    static constexpr int K = 32;
};
template <>
struct Mfma<_Float16> {
    static constexpr int K = 32;
};

// One chunk of this wave's 16x16 sub-tile for NT tau samples.  pa / pb:
// [NT][32 rows][lrow] operand panels (A rows of the P range, B rows of the Q
// range).  Every lane reads 8 consecutive K values of its row per MFMA group:
// FP32 lane group lk owns K = 8 lk + j of the chunk and feeds them to 8
// successive 16x16x4 MFMAs (a dot product does not depend on how K is split
// over the steps), so the re/im partner of every value sits in the same lane.
template <typename T, int NT>
__device__ inline void lp_chunk(const T *pa, const T *pb, int wp, int wq, f4v (&re)[NT], f4v (&im)[NT]) {
    constexpr int LR = lrow<T>();
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    typedef T v8 __attribute__((ext_vector_type(8)));
    if constexpr (Mfma<T>::K == 4) {
        for (int t = 0; t < NT; ++t) {
            const v8 a = *reinterpret_cast<const v8 *>(pa + (t * 32 + 16 * wp + li) * LR + 8 * lk);
            const v8 b = *reinterpret_cast<const v8 *>(pb + (t * 32 + 16 * wq + li) * LR + 8 * lk);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float w = (j & 1) ? b[j - 1] : -b[j + 1];  // W = (-im, re)
                re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], re[t], 0, 0, 0);
                im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], w, im[t], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int ks = 0; ks < lkc<T>(); ks += 32)
            for (int t = 0; t < NT; ++t) {
                const v8 a = *reinterpret_cast<const v8 *>(pa + (t * 32 + 16 * wp + li) * LR + ks + 8 * lk);
                const v8 b = *reinterpret_cast<const v8 *>(pb + (t * 32 + 16 * wq + li) * LR + ks + 8 * lk);
                v8 w;
                for (int c = 0; c < 4; ++c) {
                    w[2 * c] = -b[2 * c + 1];
                    w[2 * c + 1] = b[2 * c];
                }
                if constexpr (__is_same(T, __bf16)) {
                    re[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, re[t], 0, 0, 0);
                    im[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w, im[t], 0, 0, 0);
                } else {
                    re[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, re[t], 0, 0, 0);
                    im[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, w, im[t], 0, 0, 0);
                }
            }
    }
}

// Stream K in [K_lo, K_hi) (multiples of the chunk) through double-buffered LDS
// panels: every thread moves 16-byte units of the NT x (A, B) panels; the next
// chunk's loads are issued before the current chunk's MFMAs.
template <typename T, int NT>
__device__ inline void lp_stream(const T *__restrict__ U, int R, int Ktot, int rp, int rq, int K_lo, int K_hi, int t0,
                                 T *panels, f4v (&re)[NT], f4v (&im)[NT]) {
    constexpr int LKC = lkc<T>(), LR = lrow<T>();
    constexpr int UPR = LKC * (int)sizeof(T) / 16;  // 16-byte units per panel row
    constexpr int UPP = 32 * UPR;                   // units per panel
    constexpr int NU = NT * 2 * UPP;                // units per chunk
    constexpr int PER = (NU + 255) / 256;           // units per thread
    constexpr int CH = NT * 2 * 32 * LR;            // elements of T per chunk buffer
    const int tid = threadIdx.x, wave = tid >> 6, wp = wave >> 1, wq = wave & 1;
    uint4 reg[PER];
    auto gload = [&](int K0) {
        for (int j = 0; j < PER; ++j) {
            const int u = tid + 256 * j;
            if (u < NU) {
                const int t = u / (2 * UPP), ab = (u / UPP) & 1, w = u % UPP, row = w / UPR, cu = w % UPR;
                const T *src = U + (size_t)(t0 + t) * R * Ktot + (size_t)((ab ? rq : rp) + row) * Ktot + K0 +
                               cu * (16 / (int)sizeof(T));
                reg[j] = *reinterpret_cast<const uint4 *>(src);
            }
        }
    };
    auto lstore = [&](int buf) {
        for (int j = 0; j < PER; ++j) {
            const int u = tid + 256 * j;
            if (u < NU) {
                const int t = u / (2 * UPP), ab = (u / UPP) & 1, w = u % UPP, row = w / UPR, cu = w % UPR;
                T *dst = panels + buf * CH + ab * (NT * 32 * LR) + (t * 32 + row) * LR + cu * (16 / (int)sizeof(T));
                *reinterpret_cast<uint4 *>(dst) = reg[j];
            }
        }
    };
    const int n_chunks = (K_hi - K_lo) / LKC;
    if (n_chunks == 0) return;
    gload(K_lo);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < n_chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < n_chunks) gload(K_lo + (c + 1) * LKC);
        lp_chunk<T, NT>(panels + buf * CH, panels + buf * CH + NT * 32 * LR, wp, wq, re, im);
        if (c + 1 < n_chunks) lstore(buf ^ 1);
        __syncthreads();
    }
}

template <typename T, int NT, bool GRAD>
__global__ __launch_bounds__(256) void green_lp_kernel(const T *__restrict__ U, int Ko, int Ktot,
                                                       const double *__restrict__ wtau, const double *__restrict__ hinv,
                                                       const int *__restrict__ tiles, const int *__restrict__ work,
                                                       int n_slots, int R, int m, int t0, double *__restrict__ partial,
                                                       double2 *__restrict__ Hm, double2 *__restrict__ Hp,
                                                       double cgrad) {
    constexpr int PANEL_BYTES = 2 * NT * 2 * 32 * lrow<T>() * (int)sizeof(T);
    constexpr int EPI_BYTES = 4 * 512 * (int)sizeof(cplx);
    __shared__ __align__(16) unsigned char smem[PANEL_BYTES > EPI_BYTES ? PANEL_BYTES : EPI_BYTES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int item = work[blockIdx.x];
    const int slot = 4 * blockIdx.x + wave;
    if (item < 0) {  // padding block: zero partials
        if (lane == 0)
            for (int t = 0; t < NT; ++t) {
                double *out = partial + ((size_t)(t0 + t) * n_slots + slot) * 2;
                out[0] = out[1] = 0.0;
            }
        return;
    }
    const int PT = tiles[2 * item], QT = tiles[2 * item + 1];
    const int rp = 32 * PT, rq = 32 * QT;
    f4v gm_re[NT], gm_im[NT], gp_re[NT], gp_im[NT];
    for (int t = 0; t < NT; ++t) gm_re[t] = gm_im[t] = gp_re[t] = gp_im[t] = f4v{0.f, 0.f, 0.f, 0.f};
    T *panels = reinterpret_cast<T *>(smem);
    lp_stream<T, NT>(U, R, Ktot, rp, rq, 0, Ko, t0, panels, gm_re, gm_im);
    lp_stream<T, NT>(U, R, Ktot, rp, rq, Ko, Ktot, t0, panels, gp_re, gp_im);

    cplx *Gm = reinterpret_cast<cplx *>(smem) + wave * 512;
    cplx *Gp = Gm + 256;
    for (int t = 0; t < NT; ++t) {
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * lk + v;  // MFMA f32 result row of element v
            Gm[i * 16 + li] = {(double)gm_re[t][v], (double)gm_im[t][v]};
            Gp[i * 16 + li] = {(double)gp_re[t][v], (double)gp_im[t][v]};
        }
        __syncthreads();
        contract_pairs<GRAD>(Gm, Gp, PT, QT, m, hinv, wtau[t0 + t], cgrad, R,
                             partial + ((size_t)(t0 + t) * n_slots + slot) * 2,
                             GRAD ? Hm + (size_t)(t0 + t) * R * R : nullptr,
                             GRAD ? Hp + (size_t)(t0 + t) * R * R : nullptr);
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_lp_typed(const mcmp2_ctx *c, int n_tau, bool grad) {
    T *U = reinterpret_cast<T *>(c->U);
    dim3 g(c->R / 64, (c->nsp + 31) / 32, n_tau);
    lp_operands_kernel<T><<<g, 256, 0, c->stream>>>(reinterpret_cast<const float2 *>(c->psi), c->scale, c->R,
                                                    c->nsp, c->no, c->Ko, c->Ktot, U);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double cgrad = -0.5 / (0.5 * (double)c->m * (double)(c->m - 1) * (double)n_tau);
    double2 *Hm = reinterpret_cast<double2 *>(c->Hm), *Hp = reinterpret_cast<double2 *>(c->Hp);
    const int nblocks = c->n_slots / 4;
    constexpr int NTMAX = sizeof(T) == 4 ? 2 : 4;  // FP32 panels are twice as large
    for (int t0 = 0; t0 < n_tau; t0 += NTMAX) {
        const int nt = std::min(NTMAX, n_tau - t0);
#define LP_LAUNCH(NTV)                                                                                            \
    if (grad)                                                                                                     \
        green_lp_kernel<T, NTV, true><<<nblocks, 256, 0, c->stream>>>(U, c->Ko, c->Ktot, c->wtau, c->hinv,       \
                                                                      c->tiles, c->work, c->n_slots, c->R, c->m, \
                                                                      t0, c->partial, Hm, Hp, cgrad);            \
    else                                                                                                          \
        green_lp_kernel<T, NTV, false><<<nblocks, 256, 0, c->stream>>>(U, c->Ko, c->Ktot, c->wtau, c->hinv,      \
                                                                       c->tiles, c->work, c->n_slots, c->R,      \
                                                                       c->m, t0, c->partial, nullptr, nullptr,   \
                                                                       0.0)
        switch (nt) {
            case 1: LP_LAUNCH(1); break;
            case 2: LP_LAUNCH(2); break;
            case 3: LP_LAUNCH(3); break;
            default: LP_LAUNCH(4); break;
        }
#undef LP_LAUNCH
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_green_lp(const mcmp2_ctx *c, int n_tau, bool grad) {
    switch (c->precision) {
        case MCMP2_FP32: return launch_lp_typed<float>(c, n_tau, grad);
        case MCMP2_BF16: return launch_lp_typed<__bf16>(c, n_tau, grad);
        default: return launch_lp_typed<_Float16>(c, n_tau, grad);
    }
}
