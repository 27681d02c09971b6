// Low-precision Green's functions (BF16, FP16 operands on MFMA with FP32
// accumulation) followed by the pair contraction in FP32 arithmetic with FP64
// weights and sums (Sec. III of the paper: G+ / G- and the redundant-walker
// estimator).  FP32 mode runs the FP64 kernel's structure (green.hip).
//
// Operands.  For tau sample t, lp_operands writes
//   U_t[row][K] = psi[k][row] * sqrt(s_t[k]),  K = 2 k (+1 for the imaginary part),
// with s_t[k] = exp(+eps_k tau) (occupied) / exp(-eps_k tau) (virtual)
// computed and square-rooted in FP64 and rounded to FP32; psi is FP32 (the
// spinor GEMM's accumulators), so the product is formed in FP32 and rounded
// once more to the operand type (hardware FP32 -> BF16 / FP16 conversions;
// the double rounding changes a value by one operand unit in rare ties).  The symmetric square-root scaling keeps both operands within
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
#include <type_traits>

#include "contract.hpp"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

// Reals of K per LDS chunk (64 = two 16x16x32 K-steps) and the padded LDS
// row length: 16 extra bytes per row so that the 16-byte reads of 8
// consecutive rows fall in distinct banks.
template <typename T>
constexpr int lkc() {
    return 64;
}
template <typename T>
constexpr int lrow() {
    return lkc<T>() + 16 / (int)sizeof(T);
}

// FP32 -> operand type, rounded to nearest even (v_cvt_pk_bf16_f32 / v_cvt_f16_f32)
template <typename T>
__device__ inline T to_op(float v);
template <>
__device__ inline __bf16 to_op<__bf16>(float v) {
    return (__bf16)v;
}
template <>
__device__ inline _Float16 to_op<_Float16>(float v) {
    return (_Float16)v;
}

// (re, im) rounded to the operand type, packed into 32 bits (real part low)
template <typename T>
__device__ inline uint32_t pack_op(float re, float im) {
    const T a = to_op<T>(re), b = to_op<T>(im);
    return (uint32_t)__builtin_bit_cast(unsigned short, a) | ((uint32_t)__builtin_bit_cast(unsigned short, b) << 16);
}

// grid (R / 64, ceil(nsp / 32), ceil(n_tau / tpb)); psi float2 [nsp][R] ->
// U_t [R][Ktot] for tpb tau samples per block from one LDS copy of the
// block's psi tile (tpb = n_tau when the first two grid dimensions alone
// give every CU several blocks, else 1).  With gradients (V set) the same
// tile also gives the adjoint GEMM's operand V_t[k][row] = psi s_t[k] as
// packed BF16 pairs (see adjoint_lp.hip).
template <typename T>
__global__ __launch_bounds__(256) void lp_operands_kernel(const float2 *__restrict__ psi,
                                                          const double *__restrict__ scale, int R, int nsp, int no,
                                                          int Ko, int Ktot, int n_tau, int tpb, T *__restrict__ U,
                                                          uint32_t *__restrict__ V) {
    __shared__ float2 tile[32][65];
    __shared__ float sq[32], sf[32];  // sqrt(s_t[k]) and s_t[k], each rounded once from FP64
    const int r0 = 64 * blockIdx.x, k0 = 32 * blockIdx.y;
    const int t_lo = tpb * (int)blockIdx.z, t_hi = min(n_tau, t_lo + tpb);
    const int tid = threadIdx.x;
    {
        // all eight loads in flight before the first LDS store (coalesced
        // along rows; rows past nsp re-read the last spinor and store zero)
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j, kk = e >> 6, r = e & 63;
            v[j] = psi[(size_t)min(k0 + kk, nsp - 1) * R + r0 + r];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j, kk = e >> 6, r = e & 63;
            tile[kk][r] = k0 + kk < nsp ? v[j] : float2{0.f, 0.f};
        }
    }
    for (int t = t_lo; t < t_hi; ++t) {
        if (t > t_lo) __syncthreads();  // sq of the previous tau sample has been used
        if (tid < 32) {
            const int k = k0 + tid;
            const double sv = k < nsp ? scale[(size_t)t * nsp + k] : 0.0;
            sf[tid] = (float)sv;
            sq[tid] = (float)sqrt(sv);
        }
        __syncthreads();
        T *Ut = U + (size_t)t * R * Ktot;
        for (int e = tid; e < 32 * 64; e += 256) {  // coalesced along K within a row
            const int r = e >> 5, kk = e & 31, k = k0 + kk;
            if (k >= nsp) continue;
            const int K = k < no ? 2 * k : Ko + 2 * (k - no);
            const float2 v = tile[kk][r];
            // psi is FP32 (the spinor GEMM's accumulators): the products are
            // formed in FP32 and rounded once more to the operand type
            *reinterpret_cast<uint32_t *>(Ut + (size_t)(r0 + r) * Ktot + K) = pack_op<T>(v.x * sq[kk], v.y * sq[kk]);
        }
        if (V) {
            uint32_t *Vt = V + (size_t)t * nsp * R;
            for (int e = tid; e < 32 * 64; e += 256) {  // coalesced along rows
                const int kk = e >> 6, r = e & 63, k = k0 + kk;
                if (k >= nsp) continue;
                const float2 v = tile[kk][r];
                Vt[(size_t)k * R + r0 + r] = pack_op<__bf16>(v.x * sf[kk], v.y * sf[kk]);
            }
        }
    }
}

// MFMA wrappers: 16x16 output tiles, result D[4 (l / 16) + v][l % 16] in element v.
template <typename T>
struct Mfma;
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
// range).  Every lane reads 8 consecutive K values of its row per MFMA, so
// the re/im partner of every value sits in the same lane.
template <typename T, int NT>
__device__ __attribute__((always_inline)) inline void lp_chunk(const T *pa, const T *pb, int wp, int wq, f4v (&re)[NT], f4v (&im)[NT]) {
    constexpr int LR = lrow<T>();
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    typedef T v8 __attribute__((ext_vector_type(8)));
    {
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
__device__ __attribute__((always_inline)) inline void lp_stream(const T *__restrict__ U, int R, int Ktot, int rp, int rq, int K_lo, int K_hi, int t0,
                                 T *panels, f4v (&re)[NT], f4v (&im)[NT]) {
    constexpr int LKC = lkc<T>(), LR = lrow<T>();
    constexpr int UPR = LKC * (int)sizeof(T) / 16;  // 16-byte units per panel row
    constexpr int UPP = 32 * UPR;                   // units per panel
    constexpr int NU = NT * 2 * UPP;                // units per chunk
    constexpr int PER = (NU + 255) / 256;           // units per thread
    constexpr int CH = NT * 2 * 32 * LR;            // elements of T per chunk buffer
    const int tid = threadIdx.x, wave = tid >> 6, wp = wave >> 1, wq = wave & 1;
    // Loads are branch-free (a thread past the last unit re-reads the last
    // one) and the loops unrolled, so the staging registers stay registers.
    u32x4 reg[PER];  // ext_vector_type: HIP's uint4 struct defeats scalar replacement
    auto gload = [&](int K0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int u = min(tid + 256 * j, NU - 1);
            const int t = u / (2 * UPP), ab = (u / UPP) & 1, w = u % UPP, row = w / UPR, cu = w % UPR;
            const T *src = U + (size_t)(t0 + t) * R * Ktot + (size_t)((ab ? rq : rp) + row) * Ktot + K0 +
                           cu * (16 / (int)sizeof(T));
            reg[j] = *reinterpret_cast<const u32x4 *>(src);
        }
    };
    auto lstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int u = tid + 256 * j;
            if (u < NU) {
                const int t = u / (2 * UPP), ab = (u / UPP) & 1, w = u % UPP, row = w / UPR, cu = w % UPR;
                T *dst = panels + buf * CH + ab * (NT * 32 * LR) + (t * 32 + row) * LR + cu * (16 / (int)sizeof(T));
                *reinterpret_cast<u32x4 *>(dst) = reg[j];
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

// HT: element type of the adjoint blocks (FP64 complex with FP32 operands,
// packed BF16 pairs with BF16 / FP16 operands).  BREIT: the Gaunt / Breit
// interaction (one tau per block): the FP32 Green's functions are staged in
// FP64 and go through the FP64 alpha-weighted contraction of the FP64 / FP32
// modes (contract_pairs_breit; rhat [m_pad][4] unit vectors of r1p - r2p,
// gauge = weight of the second Breit term); with GRAD the kernel copies the
// pairs' G blocks into Hm / Hp as BF16 pairs for the Breit adjoint kernel
// (G-(1,3), G-(2,4) and the four G+ blocks of each pair p < q < m).
template <typename T, int NT, bool GRAD, typename HT, bool BREIT = false>
__global__ __launch_bounds__(256) void green_lp_kernel(const T *__restrict__ U, int Ko, int Ktot,
                                                       const double *__restrict__ wtau, const double *__restrict__ hinv,
                                                       const int *__restrict__ tiles, const int *__restrict__ work,
                                                       int n_slots, int R, int m, int t_base,
                                                       double *__restrict__ partial, HT *__restrict__ Hm,
                                                       HT *__restrict__ Hp, double cgrad,
                                                       const double *__restrict__ rhat = nullptr, double gauge = 0.0) {
    static_assert(!BREIT || NT == 1, "the Gaunt / Breit contraction takes one tau");
    const int t0 = t_base + (int)blockIdx.y * NT;  // tau samples t0 .. t0 + NT - 1
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
#pragma unroll  // constant indices keep the accumulators in registers
    for (int t = 0; t < NT; ++t) {
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * lk + v;  // MFMA f32 result row of element v
            Gm[i * 16 + li] = {(double)gm_re[t][v], (double)gm_im[t][v]};
            Gp[i * 16 + li] = {(double)gp_re[t][v], (double)gp_im[t][v]};
            if constexpr (GRAD && BREIT) {
                // the pair blocks p < q < m for the Breit adjoint kernel, as BF16 pairs:
                // G- only in its (1,3), (2,4) blocks (H-(1,4), H-(2,3) stay zero), all of G+
                const int row = rp + 16 * (wave >> 1) + i, col = rq + 16 * (wave & 1) + li;
                if ((row >> 3) < (col >> 3) && (col >> 3) < m) {
                    const size_t o = (size_t)(t0 + t) * R * R + (size_t)row * R + col;
                    if (((row ^ col) & 4) == 0) Hm[o] = bf16_pair(gm_re[t][v], gm_im[t][v]);
                    Hp[o] = bf16_pair(gp_re[t][v], gp_im[t][v]);
                }
            }
        }
        // wave-private staging (the K loop ended with a block barrier); one
        // wave's LDS accesses complete in order
        __builtin_amdgcn_wave_barrier();
        if constexpr (BREIT)
            contract_pairs_breit(Gm, Gp, PT, QT, m, hinv, rhat, gauge, wtau[t0 + t],
                                 partial + ((size_t)(t0 + t) * n_slots + slot) * 2);
        else  // FP32 contraction arithmetic (weights and sums in FP64)
            contract_pairs<GRAD, HT, float>(Gm, Gp, PT, QT, m, hinv, wtau[t0 + t], cgrad, R,
                                            partial + ((size_t)(t0 + t) * n_slots + slot) * 2,
                                            GRAD ? Hm + (size_t)(t0 + t) * R * R : nullptr,
                                            GRAD ? Hp + (size_t)(t0 + t) * R * R : nullptr);
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// BF16 / FP16 operands, large problems: (tau, tile pair) items with 128 x 128
// tiles (16 x 16 walkers), each run by one block of 8 waves or by two blocks
// of 4 waves (128 x 64 halves; green_big_kernel's NW), G- and G+ both kept in
// registers (each wave: 64 rows x 32 columns of each).  Work items
// (tau-major, tile pairs in 4 x 8 patches) are dealt to the XCDs in
// contiguous ranges (block b runs on XCD b % 8), so that blocks of one XCD
// share operand rows in its L2.  The epilogue stages each wave's G rows in
// LDS (FP32) two walkers at a time and runs the FP64 pair contraction.
constexpr int BW = 16;          // walkers per big tile side
constexpr int BT = 8 * BW;      // rows per big tile side
constexpr int BKW = 32;         // 32-bit words (one complex operand each) per row per chunk: one 128-B LDS row

// LDS rows of 128 B hold eight 16-byte units; unit c of row r sits at slot
// c ^ (r & 7), so 16-byte reads of one unit from 8 consecutive rows, and the
// row-wise writes of the staging, touch distinct banks (measured on gfx950 with
// the SQ_LDS_BANK_CONFLICT counter; padded 144-byte rows do conflict).
__device__ inline int swz(int row, int unit) { return row * 8 + (unit ^ (row & 7)); }

template <typename T>
__device__ inline f4v mfma_pair(u32x4 a, u32x4 b, f4v c) {
    if constexpr (__is_same(T, __bf16))
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
}

// K chunks reach LDS by direct global -> LDS loads (global_load_lds_dwordx4)
// into a ring of stages, with explicit vmcnt waits: the compiler does not
// track these loads, so it adds no waits of its own before the LDS reads.
// The loads take their LDS address in M0, which the assembly sets without
// declaring it (the compiler does not allocate M0): this relies on the
// compiled kernels using M0 for nothing else, which a CPU test checks in
// their AMD assembly (every M0 access is one of these loads or its set-up).
// The s_nop covers the wait state an M0 write needs before an LDS DMA reads it.
//
// NW = 8: one block of 8 waves per (tau, 128 x 128 tile pair), one block per
// CU.  NW = 4: the tile pair split into two 128 x 64 halves (the same
// per-wave tiles), one block of 4 waves each, two blocks per CU, so that one
// block's epilogue (FP32 / FP64 vector work) runs beside the other's MFMAs.
template <int NW>
struct BigCfg {
    static constexpr int BTB = NW == 8 ? BT : BT / 2;   // B rows (columns of the tile)
    static constexpr int STAGE = (BT + BTB) * BKW;      // words per stage: A rows then B rows
    static constexpr int DPC = (BT + BTB) / 8 / NW;     // direct loads per wave and chunk (one 8-row group each)
    static constexpr int AHEAD = NW == 8 ? 2 : 1;       // chunks in flight beyond the next one
    static constexpr int NST = AHEAD + 2;               // ring stages
};

// waits until at most k chunks (DPC direct loads each) of this wave are in flight
template <int DPC>
__device__ inline void wait_dma_chunks(int k) {
    if (k >= 2)
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * DPC) : "memory");
    else if (k == 1)
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(DPC) : "memory");
    else
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

template <typename T, bool GRAD, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2))) void green_big_kernel(
    const uint32_t *__restrict__ U, int Kow, int Ktw, const double *__restrict__ wtau,
    const double *__restrict__ hinv, const int *__restrict__ tiles16, int n_tp, int n_items, int R, int m,
    double *__restrict__ partial, uint32_t *__restrict__ Hm, uint32_t *__restrict__ Hp, double cgrad) {
    using C = BigCfg<NW>;
    constexpr int STAGE = C::STAGE, NST = C::NST, DPC = C::DPC, AHEAD = C::AHEAD, WC = NW / 2;
    __shared__ __align__(16) uint32_t lds[NST * STAGE];
    const int per = (n_items + 7) / 8;
    const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= n_items) return;
    // NW = 4: items 2 i and 2 i + 1 are the two column halves of tile-pair item i
    const int pair_item = NW == 8 ? item : item >> 1, half = NW == 8 ? 0 : item & 1;
    const int t = pair_item / n_tp, tp = pair_item % n_tp;
    const int P = tiles16[2 * tp], Q = tiles16[2 * tp + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WC, wc = wave % WC, li = lane & 15, lk = lane >> 4;
    const uint32_t *Ut = U + (size_t)t * R * Ktw;
    const int q0 = BT * Q + C::BTB * half;  // first B row

    f4v gm_re[4][2], gm_im[4][2], gp_re[4][2], gp_im[4][2];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 2; ++j) gm_re[i][j] = gm_im[i][j] = gp_re[i][j] = gp_im[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    // direct loads: wave w fills the 8-row groups g = w + NW j of a stage (A rows of P, then
    // B rows), one 16-byte unit per lane: row 8 g + lane / 8 at slot lane % 8, i.e. global
    // unit (lane % 8) ^ (row & 7) (the swizzle of swz)
    const uint32_t *dsrc[DPC];
#pragma unroll
    for (int j = 0; j < DPC; ++j) {
        const int row = 8 * (wave + NW * j) + lane / 8, unit = (lane & 7) ^ (row & 7);
        const int grow = row < BT ? BT * P + row : q0 + (row - BT);
        dsrc[j] = Ut + (size_t)min(grow, R - 1) * Ktw + 4 * unit;
    }
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)(&lds[0]);
    auto dma = [&](int w0, int st) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < DPC; ++j) {
            const uint32_t m0v =
                __builtin_amdgcn_readfirstlane(lds0 + 4u * (uint32_t)(st * STAGE) + 1024u * (uint32_t)(wave + NW * j));
            asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(m0v),
                         "v"(dsrc[j] + w0)
                         : "memory");
        }
    };
    // G(x, y) = sum_k U_x conj(U_y): Re = U_x . U_y, Im = U_x . (-Im U_y, Re U_y)
    auto rdf = [&](int st, int s, u32x4(&fa)[4], u32x4(&fb)[2]) __attribute__((always_inline)) {
        const uint32_t *l = &lds[st * STAGE];  // 16-byte units: lane group lk reads unit 4 s + lk
#pragma unroll
        for (int i = 0; i < 4; ++i)
            fa[i] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(64 * wr + 16 * i + li, 4 * s + lk));
#pragma unroll
        for (int j = 0; j < 2; ++j)
            fb[j] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(BT + 32 * wc + 16 * j + li, 4 * s + lk));
    };
    auto mmf = [&](const u32x4(&fa)[4], const u32x4(&fb)[2], f4v(&re)[4][2], f4v(&im)[4][2])
                   __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            u32x4 w;
            for (int q = 0; q < 4; ++q) w[q] = ((fb[j][q] >> 16) | (fb[j][q] << 16)) ^ 0x8000u;
            for (int i = 0; i < 4; ++i) {
                re[i][j] = mfma_pair<T>(fa[i], fb[j], re[i][j]);
                im[i][j] = mfma_pair<T>(fa[i], w, im[i][j]);
            }
        }
    };
    // One ring over the G- chunks followed by the G+ chunks (contiguous in K).
    // Each chunk holds two MFMA K steps whose fragments sit in two register
    // sets: the barrier that publishes chunk c + 1 comes between chunk c's
    // two K steps, so chunk c + 1's first fragments are read while chunk c's
    // second K step multiplies.  The stage refilled after that barrier held
    // chunk c - 1, whose reads every wave consumed before reaching it.
    const int nm = Kow / BKW, n = Ktw / BKW;
    u32x4 fa0[4], fb0[2], fa1[4], fb1[2];
    // chunk c < n - 1 (the last chunk, below, publishes nothing; a single
    // path through the step keeps the compiler's LDS-read waits exact)
    auto step = [&](int c, f4v(&re)[4][2], f4v(&im)[4][2]) __attribute__((always_inline)) {
        rdf(c % NST, 1, fa1, fb1);
        __builtin_amdgcn_sched_barrier(0);  // reads issued ahead of the MFMAs that hide them
        mmf(fa0, fb0, re, im);
        // this wave's loads of chunk c + 1 are done once only those of later chunks are out
        wait_dma_chunks<DPC>(min(AHEAD - 1, n - 2 - c));
        asm volatile("s_barrier" ::: "memory");
        if (c + AHEAD + 1 < n) dma((c + AHEAD + 1) * BKW, (c + AHEAD + 1) % NST);
        rdf((c + 1) % NST, 0, fa0, fb0);
        __builtin_amdgcn_sched_barrier(0);
        mmf(fa1, fb1, re, im);
    };
#pragma unroll
    for (int c = 0; c <= AHEAD; ++c)
        if (c < n) dma(c * BKW, c);
    wait_dma_chunks<DPC>(min(AHEAD, n - 1));
    asm volatile("s_barrier" ::: "memory");
    rdf(0, 0, fa0, fb0);
    for (int c = 0; c < nm; ++c) step(c, gm_re, gm_im);  // nm < n: G+ has at least one chunk
    for (int c = nm; c < n - 1; ++c) step(c, gp_re, gp_im);
    // the epilogue's pair weights, loaded once here (in order behind the direct loads):
    // h of walker rows 8 wr + k of P and of this lane group's column walker
    double hp[8], hq;
#pragma unroll
    for (int k = 0; k < 8; ++k) hp[k] = hinv[min(BW * P + 8 * wr + k, m - 1)];
    hq = hinv[min(q0 / 8 + 4 * wc + lk, m - 1)];
    rdf((n - 1) % NST, 1, fa1, fb1);
    __builtin_amdgcn_sched_barrier(0);
    mmf(fa0, fb0, gp_re, gp_im);
    mmf(fa1, fb1, gp_re, gp_im);
    __syncthreads();  // the epilogue reuses the stages

    // epilogue: wave-private G rows in LDS (so wave barriers order the staging
    // and the reads; the K loop ended with a block barrier), 8 rows (one walker) x 32 columns
    // (four walkers) at a time.  Rows are padded to 36 complex (288 B, i.e.
    // 32 B apart modulo the 256-byte bank row), so the 4-row reads of the
    // contraction hit each bank at most twice.
    constexpr int GLD = 36, WST = 1920;  // float2 per wave's staging slot (15 KB)
    float2 *Gm = reinterpret_cast<float2 *>(lds) + wave * WST;
    float2 *Gp = Gm + 8 * GLD;
    uint32_t *Hm_t = GRAD ? Hm + (size_t)t * R * R : nullptr;
    uint32_t *Hp_t = GRAD ? Hp + (size_t)t * R * R : nullptr;
    const double wt = wtau[t];
    double dsum = 0.0, xsum = 0.0;
    // With gradients, when every walker pair of the block counts (p < q < m),
    // the adjoint blocks are staged in the wave's LDS slot and stored in whole
    // 128-byte rows: D (8 x 32) the rows of walker p x the wave's 32 columns,
    // T (32 x 32) their Hermitian partners for four walkers p at a time.  H-'s
    // (1,4) / (2,3) blocks, which are zero, stay zero in Dm / Tm and are stored
    // with the rest.  Otherwise each element and its partner are stored apart.
    const int qb = q0 / 8 + 4 * wc;  // first column walker of the wave
    const bool staged = GRAD && P < Q && q0 / 8 + C::BTB / 8 <= m;
    uint32_t *Dm = reinterpret_cast<uint32_t *>(Gp + 8 * GLD), *Dp = Dm + 256, *Tm = Dp + 256, *Tp = Tm + 1024;
    if (staged) {
        *reinterpret_cast<u32x4 *>(Dm + 4 * lane) = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 4; ++j) *reinterpret_cast<u32x4 *>(Tm + 4 * (lane + 64 * j)) = u32x4{0u, 0u, 0u, 0u};
    }
    // the pair loop, compiled once per way of storing the adjoint blocks
    auto pairs = [&](auto st) __attribute__((always_inline)) {
        constexpr bool ST = decltype(st)::value;
#pragma unroll  // constant indices keep the accumulators in registers
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // MFMA result rows 4 lk + v of sub-tile i: walker row h holds lane groups lk = 2 h, 2 h + 1
                if ((lk >> 1) == h)
                    for (int j = 0; j < 2; ++j)
                        for (int v = 0; v < 4; ++v) {
                            const int e = (4 * (lk & 1) + v) * GLD + 16 * j + li;
                            Gm[e] = float2{gm_re[i][j][v], gm_im[i][j][v]};
                            Gp[e] = float2{gp_re[i][j][v], gp_im[i][j][v]};
                        }
                __builtin_amdgcn_wave_barrier();
                const int p = BW * P + 8 * wr + 2 * i + h, q = qb + lk;
                double dir, exc;
                AdjVals<float> av;
                contract_pair<GRAD, uint32_t, float>(Gm + 8 * lk, Gp + 8 * lk, GLD, p, q, p < q && q < m,
                                                     PairH{hp[2 * i + h], hq}, wt, cgrad, R, dir, exc,
                                                     ST ? nullptr : Hm_t, ST ? nullptr : Hp_t, ST ? &av : nullptr);
                if constexpr (ST) {
                    // element (8 p + dr, 8 qb + dc) into D, its partner (8 qb + dc, 8 pb + tc + dr) into T
                    // (Dt, Tt: Dm / Tm or Dp / Tp),
                    // scaled and rounded as the direct stores are
                    const int a = (lane & 15) >> 2, b = lane & 3, tc = 8 * ((2 * i + h) & 3);
                    auto sput = [&](uint32_t *Dt, uint32_t *Tt, int dr, int dc, cx<float> v, double scale)
                                    __attribute__((always_inline)) {
                        const float sc = (float)scale, re = v.re * sc, im = v.im * sc;
                        Dt[dr * 32 + dc] = bf16_pair(re, im);
                        Tt[dc * 32 + tc + dr] = bf16_pair(re, -im);
                    };
                    sput(Dm, Tm, a, 8 * lk + b, av.m13, av.cw);
                    sput(Dm, Tm, 4 + a, 8 * lk + 4 + b, av.m24, av.cw);
                    sput(Dp, Tp, a, 8 * lk + b, av.p13, av.cw);
                    sput(Dp, Tp, 4 + a, 8 * lk + 4 + b, av.p24, av.cw);
                    sput(Dp, Tp, a, 8 * lk + 4 + b, av.p14, -av.cw);
                    sput(Dp, Tp, 4 + a, 8 * lk + b, av.p23, -av.cw);
                    __builtin_amdgcn_wave_barrier();
                    {  // D: lane l stores row l / 8, 16-byte unit l % 8
                        const int row = lane >> 3, u = lane & 7;
                        const size_t g = (size_t)(8 * p + row) * R + 8 * qb + 4 * u;
                        *reinterpret_cast<u32x4 *>(Hm_t + g) = *reinterpret_cast<const u32x4 *>(Dm + row * 32 + 4 * u);
                        *reinterpret_cast<u32x4 *>(Hp_t + g) = *reinterpret_cast<const u32x4 *>(Dp + row * 32 + 4 * u);
                    }
                    if ((i & 1) && h == 1) {  // T complete for walkers pb .. pb + 3
                        const int pb = BW * P + 8 * wr + 4 * (i >> 1);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int row = 8 * j + (lane >> 3), u = lane & 7;
                            const size_t g = (size_t)(8 * qb + row) * R + 8 * pb + 4 * u;
                            *reinterpret_cast<u32x4 *>(Hm_t + g) =
                                *reinterpret_cast<const u32x4 *>(Tm + row * 32 + 4 * u);
                            *reinterpret_cast<u32x4 *>(Hp_t + g) =
                                *reinterpret_cast<const u32x4 *>(Tp + row * 32 + 4 * u);
                        }
                    }
                }
                const double d0 = lane_value(dir, 0), d1 = lane_value(dir, 16), d2 = lane_value(dir, 32),
                             d3 = lane_value(dir, 48);
                const double x0 = lane_value(exc, 0), x1 = lane_value(exc, 16), x2 = lane_value(exc, 32),
                             x3 = lane_value(exc, 48);
                dsum += ((d0 + d1) + d2) + d3;
                xsum += ((x0 + x1) + x2) + x3;
                __builtin_amdgcn_wave_barrier();
            }
    };
    if (staged)
        pairs(std::true_type());
    else
        pairs(std::false_type());
    if (lane == 0) {
        // eight slots per tile pair, slot 4 wr + (column group of four walkers)
        double *out = partial + ((size_t)pair_item * 8 + 4 * wr + WC * half + wc) * 2;
        out[0] = dsum;
        out[1] = xsum;
    }
}

template <typename T, int NW>
hipError_t launch_big_nw(const mcmp2_ctx *c, int n_tau, bool grad) {
    const int n_items = c->n_tp16 * n_tau * (8 / NW);
    const int per = (n_items + 7) / 8;
    const double cgrad = -0.5 / (0.5 * (double)c->m * (double)(c->m - 1) * (double)n_tau);
    const uint32_t *U = reinterpret_cast<const uint32_t *>(c->U);
    uint32_t *Hm = reinterpret_cast<uint32_t *>(c->Hm), *Hp = reinterpret_cast<uint32_t *>(c->Hp);
    if (grad)
        green_big_kernel<T, true, NW><<<8 * per, 64 * NW, 0, c->stream>>>(U, c->Ko / 2, c->Ktot / 2, c->wtau,
                                                                        c->hinv, c->tiles16, c->n_tp16, n_items,
                                                                        c->R, c->m, c->partial, Hm, Hp, cgrad);
    else
        green_big_kernel<T, false, NW><<<8 * per, 64 * NW, 0, c->stream>>>(U, c->Ko / 2, c->Ktot / 2, c->wtau,
                                                                         c->hinv, c->tiles16, c->n_tp16, n_items,
                                                                         c->R, c->m, c->partial, nullptr, nullptr,
                                                                         0.0);
    return hipGetLastError();
}

// Block shape of the large-problem kernel: 4 (two 4-wave half-tile blocks per
// tile pair, two per CU; measured faster at 512 walker pairs) or 8 (one 8-wave
// block per tile pair); both give the same results bit for bit.
constexpr int kBigWaves = 4;

template <typename T>
hipError_t launch_big_typed(const mcmp2_ctx *c, int n_tau, bool grad) {
    const int ps = prof_begin(c, MCMP2_K_GREEN_GEMM);
    hipError_t e = launch_big_nw<T, kBigWaves>(c, n_tau, grad);
    if (e != hipSuccess) return e;
    return prof_end(c, ps, MCMP2_K_GREEN_GEMM);
}

template <typename T>
hipError_t launch_lp_typed(const mcmp2_ctx *c, int n_tau, bool grad) {
    T *U = reinterpret_cast<T *>(c->U);
    const int bx = c->R / 64, by = (c->nsp + 31) / 32;
    const int tpb = bx * by >= 4 * c->n_cu ? n_tau : 1;
    dim3 g(bx, by, (n_tau + tpb - 1) / tpb);
    lp_operands_kernel<T><<<g, 256, 0, c->stream>>>(reinterpret_cast<const float2 *>(c->psi), c->scale, c->R,
                                                    c->nsp, c->no, c->Ko, c->Ktot, n_tau, tpb, U,
                                                    grad ? c->Vt : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (sizeof(T) == 2)
        if (green_big_selected(c, n_tau)) return launch_big_typed<T>(c, n_tau, grad);
    const double cgrad = -0.5 / (0.5 * (double)c->m * (double)(c->m - 1) * (double)n_tau);
    uint32_t *Hm = reinterpret_cast<uint32_t *>(c->Hm), *Hp = reinterpret_cast<uint32_t *>(c->Hp);
    const int nblocks = c->n_slots / 4;
    if (c->interaction != MCMP2_COULOMB) {
        // with gradients: the forward contraction copies the pairs' G blocks into
        // Hm / Hp, then the Breit adjoint kernel overwrites them with the adjoint
        const double gauge = c->interaction == MCMP2_BREIT ? 1.0 : 0.0;
        const int ps = prof_begin(c, MCMP2_K_GREEN_GEMM);
        if (grad)
            green_lp_kernel<T, 1, true, uint32_t, true><<<dim3(nblocks, n_tau), 256, 0, c->stream>>>(
                U, c->Ko, c->Ktot, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->m, 0, c->partial, Hm, Hp,
                cgrad, c->rhat, gauge);
        else
            green_lp_kernel<T, 1, false, uint32_t, true><<<dim3(nblocks, n_tau), 256, 0, c->stream>>>(
                U, c->Ko, c->Ktot, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->m, 0, c->partial, nullptr,
                nullptr, 0.0, c->rhat, gauge);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (grad && (e = launch_breit_adjoint_lp(c, n_tau, cgrad)) != hipSuccess) return e;
        return prof_end(c, ps, MCMP2_K_GREEN_GEMM);
    }
    constexpr int NTMAX = 4;
    for (int t0 = 0; t0 < n_tau; t0 += NTMAX) {
        const int nt = std::min(NTMAX, n_tau - t0);
#define LP_LAUNCH(NTV)                                                                                           \
    if (grad)                                                                                                    \
        green_lp_kernel<T, NTV, true, uint32_t><<<nblocks, 256, 0, c->stream>>>(                                 \
            U, c->Ko, c->Ktot, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->m, t0, c->partial, Hm,  \
            Hp, cgrad);                                                                                          \
    else                                                                                                         \
        green_lp_kernel<T, NTV, false, uint32_t><<<nblocks, 256, 0, c->stream>>>(                                \
            U, c->Ko, c->Ktot, c->wtau, c->hinv, c->tiles, c->work, c->n_slots, c->R, c->m, t0, c->partial,      \
            nullptr, nullptr, 0.0)
        const int ps = prof_begin(c, MCMP2_K_GREEN_GEMM);
        switch (nt) {
            case 1: LP_LAUNCH(1); break;
            case 2: LP_LAUNCH(2); break;
            case 3: LP_LAUNCH(3); break;
            default: LP_LAUNCH(4); break;
        }
#undef LP_LAUNCH
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if ((e = prof_end(c, ps, MCMP2_K_GREEN_GEMM)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

// The 128 x 128-tile kernel for the Coulomb interaction once it has 256 work
// items; the Gaunt / Breit interaction always takes the 32 x 32-tile kernel,
// whose epilogue layout the alpha-weighted contraction reads.
bool green_big_selected(const mcmp2_ctx *c, int n_tau) {
    return (c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16) && c->interaction == MCMP2_COULOMB &&
           c->n_tp16 * n_tau >= 256;
}

void build_big_tiles(int T16, std::vector<int> &tiles) {
    tiles.clear();
    for (int Pb = 0; Pb < T16; Pb += 4)
        for (int Qb = Pb / 8 * 8; Qb < T16; Qb += 8)
            for (int P = Pb; P < std::min(Pb + 4, T16); ++P)
                for (int Q = std::max(P, Qb); Q < std::min(Qb + 8, T16); ++Q) {
                    tiles.push_back(P);
                    tiles.push_back(Q);
                }
}

hipError_t launch_green_lp(const mcmp2_ctx *c, int n_tau, bool grad) {
    switch (c->precision) {
        case MCMP2_BF16: return launch_lp_typed<__bf16>(c, n_tau, grad);
        default: return launch_lp_typed<_Float16>(c, n_tau, grad);
    }
}
