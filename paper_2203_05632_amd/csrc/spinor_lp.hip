// Spinor values (Eq. (C) of the paper) and the coefficient gradient on BF16
// MFMAs (FP32 accumulation), used by the BF16 and FP16 modes (BF16 for its
// 8-bit exponent: basis values, coefficients and psi gradients span more than
// FP16's range).
//
// Both are real GEMMs over a K range with both operands stored row-major
// with K contiguous, so one 128 x 128-tile main loop (lp_gemm_tile) serves:
//   spinor values  psi[k][4 pt + 2 set + s] = sum_mu C[s][mu][k] chi_mu(r_pt)
//       A = Cb  [r = 4 k + 2 s + ri][mu'],  B = Xb [pt][mu'],  K = mu' of one set
//   coefficient gradient  Cbar[s][mu][k] = sum_pt chi_mu(r_pt) Psibar[k][4 pt + 2 set(mu) + s]
//       A = XTb [mu][pt],  B = PBb [set][r = 4 k + 2 s + ri][pt],  K = pt
// (ri: real / imaginary part; points padded to Ep, a multiple of 64).
//
// The spinor values feed every Green's function of the step and the
// coefficients are fixed over the run (a rounding of C is a fixed change of
// the orbitals, i.e. a bias, not noise), so the spinor GEMM runs split BF16:
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi), and
//   C X ~ C_hi X_hi + C_hi X_lo + C_lo X_hi
// (relative error about 2^-16), as one GEMM over a tripled K: per set, rows
// of Cb hold [hi | hi | lo] and rows of Xb [hi | lo | hi], each block the
// set's primitives padded to a multiple of 64 (nLp, nSp; nbp = nLp + nSp, row
// length 3 nbp).  Padding entries are zero for the context's life.
#include <algorithm>

#include "internal.hpp"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int LKW = 32;        // 32-bit words (two K values each) per row per chunk: 64 K values, one 128-B LDS row
constexpr int LBM = 128;       // block tile rows and columns

// LDS rows of 128 B hold eight 16-byte units; unit c of row r sits at slot
// c ^ (r & 7), so 16-byte reads of one unit from 8 consecutive rows, and the
// row-wise writes of the staging, touch distinct banks (measured on gfx950 with
// the SQ_LDS_BANK_CONFLICT counter; padded 144-byte rows do conflict).
__device__ inline int swz(int row, int unit) { return row * 8 + (unit ^ (row & 7)); }

template <typename T>
__device__ inline f4v mfma_lp(u32x4 a, u32x4 b, f4v c) {
    if constexpr (__is_same(T, __bf16))
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
}

// One 128 x 128 tile of D = A B^T over K in [0, K) (K a multiple of 64):
// A rows a_row0 .., B rows b_row0 .. (row-major, K contiguous, leading
// dimensions lda / ldb in elements of T; rows at or past a_rows / b_rows read
// the last valid row).  256 threads; wave (wr, wc) = (wave >> 1, wave & 1)
// owns rows 64 wr .. and columns 64 wc ..; acc[i][j] element v is D[64 wr +
// 16 i + 4 (l / 16) + v][64 wc + 16 j + l % 16].  One LDS stage (32 KB): the
// next chunk waits in registers while the current one is multiplied and is
// stored after a barrier.
template <typename T>
__device__ __attribute__((always_inline)) inline void lp_gemm_tile(const T *__restrict__ A, int lda, int a_row0,
                                                                   int a_rows, const T *__restrict__ B, int ldb,
                                                                   int b_row0, int b_rows, int K, uint32_t *lds,
                                                                   f4v (&acc)[4][4]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
    // staging unit u = tid + 256 j (j < 8): stage row u / 8, words 4 (u % 8) ..; units j < 4
    // are A rows, j >= 4 B rows (word offsets from A and B fit 32 bits)
    const uint32_t *Aw = reinterpret_cast<const uint32_t *>(A), *Bw = reinterpret_cast<const uint32_t *>(B);
    unsigned off[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int u = tid + 256 * j, row = u >> 3;
        off[j] = j < 4 ? (unsigned)min(a_row0 + row, a_rows - 1) * (unsigned)(lda / 2) + 4 * (u & 7)
                       : (unsigned)min(b_row0 + row - LBM, b_rows - 1) * (unsigned)(ldb / 2) + 4 * (u & 7);
    }
    u32x4 rg[8];
    auto gload = [&](int w0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            rg[j] = *reinterpret_cast<const u32x4 *>((j < 4 ? Aw : Bw) + off[j] + w0);
    };
    auto lstore = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = tid + 256 * j;
            *reinterpret_cast<u32x4 *>(&lds[4 * swz(u >> 3, u & 7)]) = rg[j];
        }
    };
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const int n = K / (2 * LKW);
    if (n == 0) return;
    gload(0);
    lstore();
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (c + 1 < n) gload((c + 1) * LKW);
        const uint32_t *l = lds;
#pragma unroll
        for (int ks = 0; ks < LKW / 4; ks += 4) {  // 16-byte units: lane group lk reads unit ks + lk
            u32x4 b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(LBM + 64 * wc + 16 * j + li, ks + lk));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const u32x4 a = *reinterpret_cast<const u32x4 *>(l + 4 * swz(64 * wr + 16 * i + li, ks + lk));
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma_lp<T>(a, b[j], acc[i][j]);
            }
        }
        if (c + 1 < n) {
            __syncthreads();  // every wave is done with this chunk
            lstore();
        }
        __syncthreads();
    }
}

// One 128 x 128 tile of the split product D = A_hi B_hi^T + A_hi B_lo^T +
// A_lo B_hi^T over K in [0, K) (K a multiple of 32), the hi and lo parts of
// each operand row sitting at element offsets (a_hi, a_lo), (b_hi, b_lo) of
// that row.  A stage holds 32 K values of each part side by side in one
// 128-byte LDS row (units 0-3 hi, 4-7 lo), so one K step reads four
// fragment sets for 48 MFMAs (the tripled-K form reads six for 48).  Layout
// of acc as in lp_gemm_tile.
__device__ __attribute__((always_inline)) inline void lp_split_tile(const __bf16 *__restrict__ A, int lda, int a_row0,
                                                                    int a_rows, int a_hi, int a_lo,
                                                                    const __bf16 *__restrict__ B, int ldb, int b_row0,
                                                                    int b_rows, int b_hi, int b_lo, int K,
                                                                    uint32_t *lds, f4v (&acc)[4][4]) {
    constexpr int STAGE = 2 * LBM * LKW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
    // staging unit u = tid + 256 j (j < 8): stage row u / 8 (A rows, then B rows), unit u % 8
    const uint32_t *src[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int u = tid + 256 * j, row = u >> 3, unit = u & 7;
        const bool a = row < LBM;
        const __bf16 *p = a ? A + (size_t)min(a_row0 + row, a_rows - 1) * lda
                            : B + (size_t)min(b_row0 + row - LBM, b_rows - 1) * ldb;
        const int off = unit < 4 ? (a ? a_hi : b_hi) + 8 * unit : (a ? a_lo : b_lo) + 8 * (unit - 4);
        src[j] = reinterpret_cast<const uint32_t *>(p + off);
    }
    u32x4 rg[8];
    auto gload = [&](int w0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) rg[j] = *reinterpret_cast<const u32x4 *>(src[j] + w0);
    };
    auto lstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = tid + 256 * j;
            *reinterpret_cast<u32x4 *>(&lds[buf * STAGE + 4 * swz(u >> 3, u & 7)]) = rg[j];
        }
    };
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const int n = K / 32;
    if (n == 0) return;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        const int buf = c & 1;
        if (c + 1 < n) gload((c + 1) * 16);  // 32 K values = 16 words per part
        const uint32_t *l = &lds[buf * STAGE];
        u32x4 ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ah[i] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(64 * wr + 16 * i + li, lk));
            al[i] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(64 * wr + 16 * i + li, 4 + lk));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bh[j] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(LBM + 64 * wc + 16 * j + li, lk));
            bl[j] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(LBM + 64 * wc + 16 * j + li, 4 + lk));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = mfma_lp<__bf16>(ah[i], bh[j], acc[i][j]);
                acc[i][j] = mfma_lp<__bf16>(ah[i], bl[j], acc[i][j]);
                acc[i][j] = mfma_lp<__bf16>(al[i], bh[j], acc[i][j]);
            }
        if (c + 1 < n) lstore(buf ^ 1);
        __syncthreads();
    }
}

__device__ inline void split_bf16(double v, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)(float)v;
    lo = (__bf16)(float)(v - (double)(float)hi);
}

// offset of primitive mu's first block in a split row (set L, then set S)
__device__ inline int split_base(int mu, int nL, int nLp) { return mu < nL ? mu : 3 * nLp + (mu - nL); }

// Cb[4 k + 2 s + ri][.] = part ri of C[s][mu][k] split as [hi | hi | lo]; grid (ceil(nb / 64), nsp)
__global__ __launch_bounds__(256) void coef_lp_kernel(const double2 *__restrict__ coef, int nb, int nL, int nLp,
                                                      int nSp, int nsp, __bf16 *__restrict__ Cb) {
    const int k = blockIdx.y;
    const int mu = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;  // q = 2 s + ri
    if (mu >= nb) return;
    const double2 cv = coef[((size_t)(q >> 1) * nb + mu) * nsp + k];
    __bf16 hi, lo;
    split_bf16((q & 1) ? cv.y : cv.x, hi, lo);
    const int blk = mu < nL ? nLp : nSp;
    __bf16 *o = Cb + ((size_t)4 * k + q) * 3 * (nLp + nSp) + split_base(mu, nL, nLp);
    o[0] = hi;
    o[blk] = hi;
    o[2 * blk] = lo;
}

// XT (FP64 [nb][E]) -> Xb [pt][.] split as [hi | lo | hi] (when Xb is
// given) and, for gradients, XTb [mu][pt] (row length Ep).  32 x 32 tiles
// through LDS, four elements per thread whose loads are all issued before the
// first store; grid (ceil(nb / 32), ceil(E / 32)).
__global__ __launch_bounds__(256) void x_lp_kernel(const double *__restrict__ XT, int nb, int nL, int nLp, int nSp,
                                                   int E, int Ep, __bf16 *__restrict__ Xb, __bf16 *__restrict__ XTb) {
    __shared__ double tile[32][33];
    const int mu0 = blockIdx.x * 32, pt0 = blockIdx.y * 32, tid = threadIdx.x;
    const int ldx = 3 * (nLp + nSp);
    double v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + 256 * j, mu = mu0 + (e >> 5), pt = pt0 + (e & 31);
        v[j] = (mu < nb && pt < E) ? XT[(size_t)mu * E + pt] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + 256 * j, r = e >> 5, p = e & 31, mu = mu0 + r, pt = pt0 + p;
        tile[r][p] = v[j];
        if (XTb && mu < nb && pt < E) XTb[(size_t)mu * Ep + pt] = (__bf16)(float)v[j];
    }
    if (!Xb) return;  // uniform over the block
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + 256 * j, p = e >> 5, r = e & 31, mu = mu0 + r, pt = pt0 + p;
        if (mu < nb && pt < E) {
            __bf16 hi, lo;
            split_bf16(tile[r][p], hi, lo);
            const int blk = mu < nL ? nLp : nSp;
            __bf16 *o = Xb + (size_t)pt * ldx + split_base(mu, nL, nLp);
            o[0] = hi;
            o[blk] = lo;
            o[2 * blk] = hi;
        }
    }
}

// Basis values of the step straight into the BF16 operands (the tiled spinor
// GEMM needs no FP64 copy): 32 (mu) x 32 (point) tiles, four values per
// thread, XTb [mu][pt] written along points and Xb [pt][.] split as
// [hi | lo | hi] along mu through an LDS transpose, as x_lp_kernel does from
// XT; points in [n_pts, E) are the padding walkers, zero.  The last row of
// blocks (blockIdx.y == ceil(E / 32)) computes the per-step scalars.
// grid (ceil(nb / 32), ceil(E / 32) + 1).
__global__ __launch_bounds__(256) void step_prep_lp_kernel(
    const double *__restrict__ walkers, int n_pts, int E, int Ep, int nb, int nL, int nLp, int nSp,
    const double4 *__restrict__ pgeo, const double2 *__restrict__ pnl, __bf16 *__restrict__ Xb,
    __bf16 *__restrict__ XTb, int m, const double *__restrict__ nuc, const double *__restrict__ gpar, int n_nuc,
    double Ng, double *__restrict__ hinv, double *__restrict__ rhat, const double *__restrict__ tau,
    const double *__restrict__ eps, int n_tau, int nsp, int no, double lambda, double *__restrict__ scale,
    double *__restrict__ wtau) {
    const int tid = threadIdx.x;
    if ((int)blockIdx.y == (E + 31) / 32) {
        const int i = blockIdx.x * 256 + tid;
        if (i < m + n_tau * nsp + n_tau)
            prep_scalar_item(i, walkers, m, nuc, gpar, n_nuc, Ng, hinv, rhat, tau, eps, n_tau, nsp, no, lambda,
                             scale, wtau);
        return;
    }
    __shared__ double tile[32][33];
    const int mu0 = blockIdx.x * 32, pt0 = blockIdx.y * 32;
    const int ldx = 3 * (nLp + nSp);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + 256 * j, r = e >> 5, p = e & 31, mu = mu0 + r, pt = pt0 + p;
        double v = 0.0;
        if (mu < nb && pt < n_pts)
            v = basis_value(pgeo[mu], pnl[mu], walkers[3 * pt], walkers[3 * pt + 1], walkers[3 * pt + 2]);
        tile[r][p] = v;
        if (XTb && mu < nb && pt < E) XTb[(size_t)mu * Ep + pt] = (__bf16)(float)v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + 256 * j, p = e >> 5, r = e & 31, mu = mu0 + r, pt = pt0 + p;
        if (mu < nb && pt < E) {
            __bf16 hi, lo;
            split_bf16(tile[r][p], hi, lo);
            const int blk = mu < nL ? nLp : nSp;
            __bf16 *o = Xb + (size_t)pt * ldx + split_base(mu, nL, nLp);
            o[0] = hi;
            o[blk] = lo;
            o[2 * blk] = hi;
        }
    }
}

// Work items dealt to the XCDs in contiguous ranges (block b runs on XCD b % 8).
__device__ inline int xcd_item(int n_items) {
    const int per = (n_items + 7) / 8;
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// psi[k][4 pt + 2 set + s] (float2): rows r = 4 k + 2 s + ri of Cb, columns pt
__global__ __launch_bounds__(256) void spinor_lp_kernel(const __bf16 *__restrict__ Cb, const __bf16 *__restrict__ Xb,
                                                        int nsp, int nLp, int nSp, int E, int R, int n_rt, int n_ct,
                                                        float2 *__restrict__ psi) {
    __shared__ __align__(16) uint32_t lds[2 * 2 * LBM * LKW];
    int set, rest;
    if (!spinor_set_item(n_rt * n_ct, set, rest)) return;
    const int rt = rest / n_ct, ct = rest % n_ct;
    // per set, Cb rows hold [hi | hi | lo] and Xb rows [hi | lo | hi]: A_hi, A_lo
    // are blocks 0 and 2 of Cb, B_hi, B_lo blocks 0 and 1 of Xb
    const int koff = set ? 3 * nLp : 0, blk = set ? nSp : nLp, ld = 3 * (nLp + nSp);
    f4v acc[4][4];
    lp_split_tile(Cb, ld, LBM * rt, 4 * nsp, koff, koff + 2 * blk, Xb, ld, LBM * ct, E, koff, koff + blk, blk, lds,
                  acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = (LBM * rt + 64 * wr + 16 * i) / 4 + lk;  // rows 4 k + v, v = 2 s + ri
        if (k >= nsp) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pt = LBM * ct + 64 * wc + 16 * j + li;
            if (pt >= E) continue;
            float2 *o = psi + (size_t)k * R + 4 * pt + 2 * set;
            o[0] = float2{acc[i][j][0], acc[i][j][1]};  // alpha
            o[1] = float2{acc[i][j][2], acc[i][j][3]};  // beta
        }
    }
}

// grad_coeffs[s][mu][k] (double2): rows mu of one set (XTb), columns r = 4 k + 2 s + ri (PBb[set]).
// The tile goes through LDS in two halves of 64 rows (rows of CGR floats: the
// 4-row steps of the MFMA result layout fall in different banks) so that the
// stores run along k: 32 consecutive complex values (512 B) per (s, mu).  With
// one 32 KB main-loop stage and a 33 KB half tile, three blocks share a CU
// (the register count, 156, allows three waves per SIMD; two blocks fit with a
// full tile), so the epilogues' HBM traffic overlaps other blocks' main loops.
constexpr int CGR = 132;
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void coef_grad_lp_kernel(
    const __bf16 *__restrict__ XTb, const __bf16 *__restrict__ PBb, int nb, int nL, int nsp, int Ep, int n_rt_L,
    int n_rt_S, int n_ct, double *__restrict__ grad_coeffs, double *__restrict__ sum, double *__restrict__ comp) {
    constexpr int MAIN = 2 * LBM * LKW, EPI = (LBM / 2) * CGR;
    __shared__ __align__(16) uint32_t lds[MAIN > EPI ? MAIN : EPI];
    const int n_items = (n_rt_L + n_rt_S) * n_ct;
    const int item = xcd_item(n_items);
    if (item >= n_items) return;
    const int rt_all = item / n_ct, ct = item % n_ct;
    const int set = rt_all >= n_rt_L;
    const int mu_lo = set ? nL : 0, mu_hi = set ? nb : nL;
    const int mu0 = mu_lo + LBM * (set ? rt_all - n_rt_L : rt_all);
    f4v acc[4][4];
    lp_gemm_tile<__bf16>(XTb, Ep, mu0, mu_hi, PBb + (size_t)set * 4 * nsp * Ep, Ep, LBM * ct, 4 * nsp, Ep, lds, acc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
    float *tile = reinterpret_cast<float *>(lds);  // [mu - mu0 - 64 h][r - LBM ct]
    const int k0 = (LBM * ct) / 4;
    // complex value e = tid + 256 q of a half: row e / 64, spin s = (e / 32) % 2, k = k0 + e % 32
    constexpr int NQ = (LBM / 2) * 64 / 256;
    constexpr int QB = 4;  // running sums loaded per batch before any is updated
    for (int h = 0; h < 2; ++h) {
        // the main loop's (or the previous half's) LDS reads are done: lp_gemm_tile
        // ends with a barrier, and so does every half
        if (wr == h) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        tile[(16 * i + 4 * lk + v) * CGR + 64 * wc + 16 * j + li] = acc[i][j][v];
        }
        __syncthreads();
        const int muh = mu0 + 64 * h;
        if (!sum) {
            for (int q = 0; q < NQ; ++q) {
                const int e = tid + 256 * q, row = e >> 6, sp = (e >> 5) & 1, kk = e & 31;
                const int mu = muh + row, k = k0 + kk;
                if (mu >= mu_hi || k >= nsp) continue;
                const float *src = tile + row * CGR + 4 * kk + 2 * sp;
                *reinterpret_cast<double2 *>(grad_coeffs + (((size_t)sp * nb + mu) * nsp + k) * 2) =
                    double2{(double)src[0], (double)src[1]};
            }
        } else {
            // Compensated accumulation instead of the store.  The running sums
            // of QB values are loaded before any of them is updated (values out
            // of range load element 0 and are not written back); each element
            // still takes one Neumaier step.
#pragma unroll 1
            for (int q0 = 0; q0 < NQ; q0 += QB) {
                size_t o[QB];
                bool ok[QB];
                double2 sv[QB], cv[QB];
#pragma unroll
                for (int u = 0; u < QB; ++u) {
                    const int e = tid + 256 * (q0 + u), row = e >> 6, sp = (e >> 5) & 1, kk = e & 31;
                    const int mu = muh + row, k = k0 + kk;
                    ok[u] = mu < mu_hi && k < nsp;
                    o[u] = ok[u] ? (((size_t)sp * nb + mu) * nsp + k) * 2 : 0;
                    sv[u] = *reinterpret_cast<const double2 *>(sum + o[u]);
                    cv[u] = *reinterpret_cast<const double2 *>(comp + o[u]);
                }
#pragma unroll
                for (int u = 0; u < QB; ++u) {
                    if (!ok[u]) continue;
                    const int e = tid + 256 * (q0 + u), row = e >> 6, sp = (e >> 5) & 1, kk = e & 31;
                    const float *src = tile + row * CGR + 4 * kk + 2 * sp;
                    neumaier(sv[u].x, cv[u].x, (double)src[0]);
                    neumaier(sv[u].y, cv[u].y, (double)src[1]);
                    *reinterpret_cast<double2 *>(sum + o[u]) = sv[u];
                    *reinterpret_cast<double2 *>(comp + o[u]) = cv[u];
                }
            }
        }
        __syncthreads();  // the half's LDS reads are done before the next half is written
    }
}

}  // namespace

hipError_t launch_coef_lp(const mcmp2_ctx *c) {
    dim3 g((c->nb + 63) / 64, c->nsp);
    coef_lp_kernel<<<g, 256, 0, c->stream>>>(reinterpret_cast<const double2 *>(c->coef), c->nb, c->nL, c->nLp,
                                             c->nbp - c->nLp, c->nsp, reinterpret_cast<__bf16 *>(c->Cb));
    return hipGetLastError();
}

// Measured on both sides of the threshold (conversion of the basis values
// included): 44 tiles (340 spinors, 256 points) took 34 us against 16 us on
// the FP32 path; 248 tiles (980 spinors, 512 points) took 68 us against 173 us.
bool spinor_lp_tiled(const mcmp2_ctx *c) {
    const int n_rt = (4 * c->nsp + LBM - 1) / LBM, n_ct = (c->E + LBM - 1) / LBM;
    return 2 * 2 * n_rt * n_ct >= c->n_cu;
}

hipError_t launch_x_lp(const mcmp2_ctx *c, bool want_xb) {
    if (!want_xb && !c->XTb) return hipSuccess;
    dim3 g((c->nb + 31) / 32, (c->E + 31) / 32);
    x_lp_kernel<<<g, 256, 0, c->stream>>>(c->XT, c->nb, c->nL, c->nLp, c->nbp - c->nLp, c->E, c->Ep,
                                          want_xb ? reinterpret_cast<__bf16 *>(c->Xb) : nullptr,
                                          reinterpret_cast<__bf16 *>(c->XTb));
    return hipGetLastError();
}

hipError_t launch_step_prep_lp(const mcmp2_ctx *c, const double *walkers, const double *tau, int n_tau) {
    const int n_items = c->m + n_tau * c->nsp + n_tau;
    const int bx = std::max((c->nb + 31) / 32, (n_items + 255) / 256);
    dim3 g(bx, (c->E + 31) / 32 + 1);
    step_prep_lp_kernel<<<g, 256, 0, c->stream>>>(
        walkers, 2 * c->m, c->E, c->Ep, c->nb, c->nL, c->nLp, c->nbp - c->nLp,
        reinterpret_cast<const double4 *>(c->pgeo), reinterpret_cast<const double2 *>(c->pnl),
        reinterpret_cast<__bf16 *>(c->Xb), reinterpret_cast<__bf16 *>(c->XTb), c->m, c->nuc, c->gpar, c->n_nuc,
        c->Ng, c->hinv, c->rhat, tau, c->eps, n_tau, c->nsp, c->no, c->lambda, c->scale, c->wtau);
    return hipGetLastError();
}

// Xb (and XTb) were written by step_prep_lp_kernel in the same step.
hipError_t launch_spinor_lp(const mcmp2_ctx *c) {
    const int n_rt = (4 * c->nsp + LBM - 1) / LBM, n_ct = (c->E + LBM - 1) / LBM;
    spinor_lp_kernel<<<16 * ((n_rt * n_ct + 7) / 8), 256, 0, c->stream>>>(
        reinterpret_cast<const __bf16 *>(c->Cb), reinterpret_cast<const __bf16 *>(c->Xb), c->nsp, c->nLp,
        c->nbp - c->nLp, c->E, c->R, n_rt, n_ct, reinterpret_cast<float2 *>(c->psi));
    return hipGetLastError();
}

// The fused accumulation reads and rewrites the running sums in the epilogue;
// with fewer than two tiles per CU those dependent loads are not hidden (340
// spinors: 66 tiles, 23 us against 8 us plus two 5 us accumulation launches).
bool coef_grad_lp_fused(const mcmp2_ctx *c) {
    const int n_rt_L = (c->nL + LBM - 1) / LBM, n_rt_S = (c->nS + LBM - 1) / LBM;
    const int n_ct = (4 * c->nsp + LBM - 1) / LBM;
    return (n_rt_L + n_rt_S) * n_ct >= 2 * c->n_cu;
}

// PBb (the psi gradient as BF16, points contiguous) was written by the
// adjoint GEMM of the same step (adjoint_lp.hip).
hipError_t launch_coef_grad_lp(const mcmp2_ctx *c, grad_out grad_coeffs) {
    const int n_rt_L = (c->nL + LBM - 1) / LBM, n_rt_S = (c->nS + LBM - 1) / LBM;
    const int n_ct = (4 * c->nsp + LBM - 1) / LBM;
    const int n_items = (n_rt_L + n_rt_S) * n_ct;
    // lp_gemm_tile addresses its operand rows by 32-bit word offsets
    if ((size_t)std::max(c->nb, 4 * c->nsp) * (size_t)(c->Ep / 2) >= ((size_t)1 << 32)) return hipErrorInvalidValue;
    coef_grad_lp_kernel<<<8 * ((n_items + 7) / 8), 256, 0, c->stream>>>(
        reinterpret_cast<const __bf16 *>(c->XTb), reinterpret_cast<const __bf16 *>(c->PBb), c->nb, c->nL, c->nsp,
        c->Ep, n_rt_L, n_rt_S, n_ct, grad_coeffs.out, grad_coeffs.sum, grad_coeffs.comp);
    return hipGetLastError();
}
