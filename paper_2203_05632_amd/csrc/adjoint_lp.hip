// Adjoint GEMM of the Green's functions with BF16 operands on MFMA (FP32
// accumulation), used by the BF16 and FP16 modes with gradients.
//
// With G_t = Psi S_t Psi^H (Sec. III of the paper: G- over occupied, G+ over
// virtual spinors; S_t = diag(exp(+eps tau_t)) or diag(exp(-eps tau_t))) and
// H_t = Gbar_t + Gbar_t^H the adjoint blocks left by the Green's-function
// kernel,
//   Psibar = sum_t H_t V_t,   V_t = Psi S_t,
//   epsbar_k = (1/2) sum_t (+-tau_t) Re(psi_k^H (H_t V_t)_k).
// All tau samples form one GEMM with K = n_tau R: A = [H_1 .. H_T] (rows x),
// B = [V_1; ..; V_T] stored as V_t[k][y] (y contiguous).  epsbar needs the
// per-tau products; the kernel keeps only the running sum over tau, so at
// each tau boundary it forms D_t[k] = Re(psi_k^H (sum_{t' <= t} H_t' V_t')_k)
// and takes D_t - D_{t-1}.
//
// Complex numbers are BF16 pairs packed in 32 bits (real part low).  With
// re/im interleaved along K, P = A B^T is two real GEMMs over the same A:
//   Re P = A . (Vr, -Vi),   Im P = A . (Vi, Vr),
// both B variants formed from one B fragment in registers (a sign flip of
// the high halves, a swap of the halves).
#include <algorithm>

#include "internal.hpp"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int AK = 32;    // complex K values (y) per LDS chunk: one 128-B LDS row
constexpr int ABM = 128;  // rows x per block (two row waves of 64)

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// LDS rows of 128 B hold eight 16-byte units; unit c of row r sits at slot
// c ^ (r & 7), so 16-byte reads of one unit from 8 consecutive rows, and the
// row-wise writes of the staging, touch distinct banks (measured on gfx950 with
// the SQ_LDS_BANK_CONFLICT counter; padded 144-byte rows do conflict).
__device__ inline int swz(int row, int unit) { return row * 8 + (unit ^ (row & 7)); }

// One block: rows [x0, x0 + 128) x spinor columns [k0, k0 + NCW WN) of one
// kind (occupied: A = H-, virtual: A = H+), 2 x NCW waves.  Waves (wr, wc)
// own 64 rows x WN columns; the lane's 16x16 sub-tiles (i, j) hold rows
// x0 + 64 wr + 16 i + 4 (l / 16) + v and column k0 + WN wc + 16 j + l % 16 in
// element v.  Wider blocks (NCW = 4) read each H row panel for twice the
// columns, halving the H traffic per flop.
// Work items (row tile, column tile), row-tile major, are dealt to the XCDs
// in contiguous ranges (block b runs on XCD b % 8), so that blocks sharing
// H rows or V columns run side by side on one L2.
// DMA: chunks go from global memory straight into a ring of three LDS stages
// (global_load_lds_dwordx4, issued two chunks ahead; no staging registers),
// waited for with an explicit vmcnt: the compiler does not track these loads,
// so it inserts no wait of its own before the LDS reads (with the load builtin
// it waits for every outstanding load there).  Vector-memory loads complete in
// issue order, so a wait the compiler places for its own later loads also
// covers these.
// The loads take their LDS address in M0, which the assembly sets without
// declaring it (the compiler does not allocate M0): this relies on the
// compiled kernels using M0 for nothing else, which a CPU test checks in
// their AMD assembly (every M0 access is one of these loads or its set-up).
// The s_nop covers the wait state an M0 write needs before an LDS DMA reads it.
template <int WN, int NCW, bool DMA>
__global__ __launch_bounds__(128 * NCW) void adj_lp_kernel(
    const uint32_t *__restrict__ Hm, const uint32_t *__restrict__ Hp, const uint32_t *__restrict__ V,
    const float2 *__restrict__ psi, const double *__restrict__ tau, int n_tau, int R, int no, int nsp,
    int n_occ_tiles, int n_col_tiles, int n_items, int Ep, unsigned short *__restrict__ PBb,
    double *__restrict__ eps_part) {
    constexpr int NTH = 128 * NCW, BN = NCW * WN, NJ = WN / 16;
    constexpr int NA = ABM * (AK / 4) / NTH;  // 16-byte A units per thread per chunk
    constexpr int NB = BN * (AK / 4) / NTH;   // 16-byte B units per thread per chunk
    constexpr int NST = DMA ? 3 : 2;
    __shared__ __align__(16) uint32_t lds[NST][(ABM + BN) * AK];
    __shared__ float dpart[2][BN];

    const int per = (n_items + 7) / 8;
    const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= n_items) return;
    const int rt = item / n_col_tiles, ct = item % n_col_tiles;
    const bool occ = ct < n_occ_tiles;
    const int k0 = occ ? BN * ct : no + BN * (ct - n_occ_tiles);
    const int k_hi = occ ? no : nsp;
    const uint32_t *H = occ ? Hm : Hp;
    const int x0 = ABM * rt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / NCW, wc = wave % NCW, li = lane & 15, lk = lane >> 4;

    // global -> register staging: unit u = tid + NTH j covers row u / 8, words 4 (u % 8) .. + 3
    const uint32_t *asrc[NA];
    const uint32_t *bsrc[NB];
    for (int j = 0; j < NA; ++j) {
        const int u = tid + NTH * j;
        asrc[j] = H + (size_t)min(x0 + u / 8, R - 1) * R + 4 * (u % 8);
    }
    for (int j = 0; j < NB; ++j) {
        const int u = tid + NTH * j;
        bsrc[j] = V + (size_t)min(k0 + u / 8, k_hi - 1) * R + 4 * (u % 8);
    }
    const size_t RR = (size_t)R * R, NR = (size_t)nsp * R;
    const int cpt = R / AK;  // chunks per tau sample
    const int n_chunks = n_tau * cpt;
    u32x4 ra[NA], rb[NB];
    auto gload = [&](u32x4(&xa)[NA], u32x4(&xb)[NB], int c) __attribute__((always_inline)) {
        const int t = c / cpt, y0 = (c % cpt) * AK;
        for (int j = 0; j < NA; ++j) xa[j] = *reinterpret_cast<const u32x4 *>(asrc[j] + t * RR + y0);
        for (int j = 0; j < NB; ++j) xb[j] = *reinterpret_cast<const u32x4 *>(bsrc[j] + t * NR + y0);
    };
    auto lstore = [&](const u32x4(&xa)[NA], const u32x4(&xb)[NB], int buf) __attribute__((always_inline)) {
        for (int j = 0; j < NA; ++j) {
            const int u = tid + NTH * j;
            *reinterpret_cast<u32x4 *>(&lds[buf][4 * swz(u / 8, u % 8)]) = xa[j];
        }
        for (int j = 0; j < NB; ++j) {
            const int u = tid + NTH * j;
            *reinterpret_cast<u32x4 *>(&lds[buf][4 * swz(ABM + u / 8, u % 8)]) = xb[j];
        }
    };

    f4v pre[4][NJ], pim[4][NJ];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < NJ; ++j) pre[i][j] = pim[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    double d_prev = 0.0, e_acc = 0.0;  // threads tid < BN: column k0 + tid
    const double sgn = occ ? 0.5 : -0.5;

    auto compute = [&](int buf) __attribute__((always_inline)) {
        const uint32_t *l = lds[buf];
#pragma unroll
        for (int ks = 0; ks < AK / 4; ks += 4) {  // 16-byte units: lane group lk reads unit ks + lk
            u32x4 a[4];
            for (int i = 0; i < 4; ++i)
                a[i] = *reinterpret_cast<const u32x4 *>(l + 4 * swz(64 * wr + 16 * i + li, ks + lk));
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const u32x4 b = *reinterpret_cast<const u32x4 *>(l + 4 * swz(ABM + WN * wc + 16 * j + li, ks + lk));
                u32x4 br, bi;
                for (int q = 0; q < 4; ++q) {
                    br[q] = b[q] ^ 0x80000000u;             // (Vr, -Vi)
                    bi[q] = (b[q] >> 16) | (b[q] << 16);    // (Vi, Vr)
                }
                for (int i = 0; i < 4; ++i) {
                    pre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[i]), as_bf16x8(br), pre[i][j], 0,
                                                                        0, 0);
                    pim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[i]), as_bf16x8(bi), pim[i][j], 0,
                                                                        0, 0);
                }
            }
        }
    };
    // after chunk c: at a tau boundary, D_t[k] over this block's rows from the running sums
    auto tau_boundary = [&](int c) __attribute__((always_inline)) {
        if ((c + 1) % cpt != 0) return;
        const int t = c / cpt;
        for (int j = 0; j < NJ; ++j) {
            const int k = k0 + WN * wc + 16 * j + li;
            float d = 0.f;
            if (k < k_hi)
                for (int i = 0; i < 4; ++i) {
                    const int xb = x0 + 64 * wr + 16 * i + 4 * lk;
                    for (int v = 0; v < 4; ++v)
                        if (xb + v < R) {
                            const float2 p = psi[(size_t)k * R + xb + v];
                            d += p.x * pre[i][j][v] + p.y * pim[i][j][v];
                        }
                }
            d += __shfl_xor(d, 16, 64);
            d += __shfl_xor(d, 32, 64);
            if (lk == 0) dpart[wr][WN * wc + 16 * j + li] = d;
        }
        __syncthreads();
        if (tid < BN) {
            const double D = (double)dpart[0][tid] + (double)dpart[1][tid];
            e_acc += sgn * tau[t] * (D - d_prev);
            d_prev = D;
        }
    };

    if constexpr (DMA) {
        // wave w fills the 8-row groups g = w + NW j of a stage, one 16-byte unit
        // per lane: row 8 g + lane / 8 at slot lane % 8, i.e. global unit
        // (lane % 8) ^ (row & 7) (the swizzle of swz)
        constexpr int NW = 2 * NCW, NG = (ABM + BN) / 8 / NW, NGA = ABM / 8 / NW;
        static_assert((ABM + BN) % (8 * NW) == 0 && ABM % (8 * NW) == 0, "row groups per wave");
        constexpr uint32_t STAGE = (ABM + BN) * AK * 4;
        const uint32_t *dsrc[NG];
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int row = 8 * (wave + NW * j) + lane / 8, unit = (lane & 7) ^ (row & 7);
            dsrc[j] = j < NGA ? H + (size_t)min(x0 + row, R - 1) * R + 4 * unit
                              : V + (size_t)min(k0 + row - ABM, k_hi - 1) * R + 4 * unit;
        }
        const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)(&lds[0][0]);
        auto dma = [&](int c) __attribute__((always_inline)) {
            const int t = c / cpt, y0 = (c % cpt) * AK;
            const uint32_t base = lds0 + (uint32_t)(c % 3) * STAGE;
#pragma unroll
            for (int j = 0; j < NG; ++j) {
                const uint32_t *g = dsrc[j] + (j < NGA ? t * RR : t * NR) + y0;
                const uint32_t m0v = __builtin_amdgcn_readfirstlane(base + 1024u * (uint32_t)(wave + NW * j));
                asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(m0v), "v"(g)
                             : "memory");
            }
        };
        dma(0);
        if (n_chunks > 1) dma(1);
        for (int c = 0; c < n_chunks; ++c) {
            // this wave's loads of chunk c are done once at most the NG of chunk c + 1 are out
            if (c + 1 < n_chunks)
                asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NG) : "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();  // every wave's chunk c is in LDS and every wave is done with chunk c - 1
            if (c + 2 < n_chunks) dma(c + 2);  // into the stage chunk c - 1 used
            compute(c % 3);
            tau_boundary(c);
        }
        __syncthreads();
    } else {
        gload(ra, rb, 0);
        lstore(ra, rb, 0);
        __syncthreads();
        for (int c = 0; c < n_chunks; ++c) {
            const int buf = c & 1;
            if (c + 1 < n_chunks) gload(ra, rb, c + 1);
            compute(buf);
            if (c + 1 < n_chunks) lstore(ra, rb, buf ^ 1);
            tau_boundary(c);
            __syncthreads();
        }
    }

    // Psibar tile -> the coefficient gradient's BF16 operand PBb[set][4 k + 2 s + ri][pt]
    // (points contiguous; row x = 4 pt + 2 set + s), one wave column (WN spinors) at a
    // time through LDS: stg[kk][2 set + s][ri][32 points], spinor rows padded to 528 bytes
    // (16-byte aligned reads; the 16 spinors a wave writes fall in distinct banks).
    constexpr int SR = 264;  // bf16 per staged spinor
    unsigned short *stg = reinterpret_cast<unsigned short *>(&lds[0][0]);
    const int pt0 = x0 / 4, n_pt = min(32, (R - x0) / 4);  // R - x0 is a multiple of 64
    const size_t plane = (size_t)4 * nsp * Ep;
    for (int g = 0; g < NCW; ++g) {
        if (wc == g) {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        unsigned short *o = stg + (16 * j + li) * SR + 2 * v * 32 + 16 * wr + 4 * i + lk;
                        o[0] = __builtin_bit_cast(unsigned short, (__bf16)pre[i][j][v]);
                        o[32] = __builtin_bit_cast(unsigned short, (__bf16)pim[i][j][v]);
                    }
        }
        __syncthreads();
        for (int e = tid; e < WN * 8 * 4; e += NTH) {  // spinor kk, staged row (2 set + s) * 2 + ri, 8 points
            const int kk = e >> 5, row = (e >> 2) & 7, unit = e & 3;
            const int k = k0 + WN * g + kk;
            if (k >= k_hi || 8 * unit >= n_pt) continue;
            const int set = row >> 2, sri = row & 3;  // sri = 2 s + ri
            *reinterpret_cast<u32x4 *>(PBb + set * plane + (size_t)(4 * k + sri) * Ep + pt0 + 8 * unit) =
                *reinterpret_cast<const u32x4 *>(stg + kk * SR + row * 32 + 8 * unit);
        }
        __syncthreads();  // the staging is rewritten for the next wave column
    }
    if (tid < BN && k0 + tid < k_hi) eps_part[(size_t)rt * nsp + k0 + tid] = e_acc;
}

template <int WN, int NCW, bool DMA = false>
hipError_t launch_adj_typed(const mcmp2_ctx *c, const double *tau, int n_tau) {
    constexpr int BN = NCW * WN;
    const int n_occ_tiles = (c->no + BN - 1) / BN, n_vir_tiles = (c->nsp - c->no + BN - 1) / BN;
    const int n_col_tiles = n_occ_tiles + n_vir_tiles;
    const int n_row_tiles = (c->R + ABM - 1) / ABM;
    const int n_items = n_row_tiles * n_col_tiles;
    const int per = (n_items + 7) / 8;
    const int ps = prof_begin(c, MCMP2_K_ADJ_GEMM);
    adj_lp_kernel<WN, NCW, DMA><<<8 * per, 128 * NCW, 0, c->stream>>>(
        reinterpret_cast<const uint32_t *>(c->Hm), reinterpret_cast<const uint32_t *>(c->Hp), c->Vt,
        reinterpret_cast<const float2 *>(c->psi), tau, n_tau, c->R, c->no, c->nsp, n_occ_tiles, n_col_tiles, n_items,
        c->Ep, reinterpret_cast<unsigned short *>(c->PBb), c->eps_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return prof_end(c, ps, MCMP2_K_ADJ_GEMM);
}

}  // namespace

int adjoint_lp_row_tiles(const mcmp2_ctx *c) { return (c->R + ABM - 1) / ABM; }

// V_t (psi s_t as packed BF16 pairs) was written by the operand kernel of the
// Green's functions in the same step (green_lp.hip).
hipError_t launch_adjoint_lp(const mcmp2_ctx *c, const double *tau, int n_tau) {
    // 128-column tiles once they give every CU a block (the 512-pair workload:
    // 416 tiles, 1028 us against 1186 us with 64-column tiles); below that the
    // narrower tiles' extra blocks win (128 pairs: 32 tiles, 101 against 67 us)
    const int wide_items = ((c->R + ABM - 1) / ABM) * ((c->no + 127) / 128 + (c->nsp - c->no + 127) / 128);
    const int wider_items = ((c->R + ABM - 1) / ABM) * ((c->no + 255) / 256 + (c->nsp - c->no + 255) / 256);
    if (4 * wider_items >= 3 * c->n_cu) return launch_adj_typed<64, 4, true>(c, tau, n_tau);
    return wide_items >= c->n_cu ? launch_adj_typed<64, 2>(c, tau, n_tau) : launch_adj_typed<32, 2>(c, tau, n_tau);
}
