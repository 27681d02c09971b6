// Spinor values at the walker positions (Sec. II, Eq. (C) of the paper):
//   phi_k^{L s}(r) = sum_{mu in L} C[s][mu][k] chi_mu(r),
//   phi_k^{S s}(r) = sum_{mu in S} C[s][mu][k] chi_mu(r),
// for the 2m electron positions of a step, where chi_mu is a Cartesian
// primitive N (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-zeta |r-A|^2).
//
// Two kernels:
//   step_prep    -- XT[mu][pt] = chi_mu(r_pt) (FP64, point index fastest),
//                   plus the per-step scalars the Green's-function kernel
//                   needs: N_g / (g(r1p) g(r2p)) and the unit vector of
//                   r1p - r2p per walker, the tau scalings
//                   exp(+eps_i tau) / exp(-eps_a tau) and w(tau);
//   spinor_gemm  -- psi[k][4 pt + c] (complex), a real x complex GEMM on
//                   FP64 MFMA (v_mfma_f64_16x16x4f64).
// (Generating the basis values inside the GEMM was measured slower: the FP64
// exp then sits on the critical path of every MFMA.)
//
// psi is stored spinor-major with the row index r = 4 pt + c = 8 p + 4 e + c
// (pair p, electron e, component c in L alpha, L beta, S alpha, S beta)
// fastest, so that a 16-row slice for one spinor is 256 contiguous bytes:
// this is the operand layout the Green's-function kernel streams.
#include "internal.hpp"

namespace {

// grid (ceil(n_pts / 128), nb + 1): rows y < nb evaluate basis function y at
// every point; row y == nb runs a grid-stride loop over the walker factors,
// the tau scalings and the tau weights.
__global__ __launch_bounds__(128) void step_prep_kernel(
    const double *__restrict__ walkers, int n_pts, int E, int nb, const double4 *__restrict__ pgeo,
    const double2 *__restrict__ pnl, double *__restrict__ XT, int m, const double *__restrict__ nuc,
    const double *__restrict__ gpar, int n_nuc, double Ng, double *__restrict__ hinv, double *__restrict__ rhat,
    const double *__restrict__ tau,
    const double *__restrict__ eps, int n_tau, int nsp, int no, double lambda, double *__restrict__ scale,
    double *__restrict__ wtau) {
    const int mu = blockIdx.y;
    if (mu < nb) {
        const int pt = blockIdx.x * blockDim.x + threadIdx.x;
        if (pt < n_pts)
            XT[(size_t)mu * E + pt] =
                basis_value(pgeo[mu], pnl[mu], walkers[3 * pt], walkers[3 * pt + 1], walkers[3 * pt + 2]);
        return;
    }
    const int n_items = m + n_tau * nsp + n_tau;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x)
        prep_scalar_item(i, walkers, m, nuc, gpar, n_nuc, Ng, hinv, rhat, tau, eps, n_tau, nsp, no, lambda, scale,
                         wtau);
}

// Small problems (too few 16-spinor x 64-point tiles to fill the GPU):
// one block computes a 16 (spinor k) x 16 (point) tile of one component set
// (blockIdx.z: 0 = L, 1 = S) for both spins, re and im: four 16x16 FP64
// accumulators.  The 4 waves split the mu range (every 4th group of 4) and
// wave 0 adds the partial tiles in a fixed order.  All loads are
// unconditional (indices clamped, values masked) so the next K-step's loads
// stay in flight across the current MFMAs.  MFMA operand layout (16x16x4
// f64): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the result
// D[4 v + l / 16][l % 16] sits in element v of the lane's accumulator
// (checked on gfx950).
//
// T = double: FP64 MFMA, psi double2.  T = float: v_mfma_f32_16x16x4f32 on
// operands rounded from FP64, FP32 accumulation, psi float2 (the operand
// source of the low-precision Green's-function kernels); its result element v
// sits at D[4 (l / 16) + v][l % 16].
template <typename T>
__global__ __launch_bounds__(256) void spinor_gemm_kernel(const double *__restrict__ XT,
                                                          const double *__restrict__ coef, int E, int nb, int nL,
                                                          int nsp, int R, void *__restrict__ psi_out) {
    typedef T acc_t __attribute__((ext_vector_type(4)));
    __shared__ acc_t red[3][4][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int set = blockIdx.z;
    const int k0 = blockIdx.x * 16;
    const int pt0 = blockIdx.y * 16;
    const int mu_lo = set == 0 ? 0 : nL;
    const int mu_hi = set == 0 ? nL : nb;
    const int li = lane & 15, lk = lane >> 4;
    const int k = k0 + li;
    const int kc = min(k, nsp - 1);
    const bool k_ok = k < nsp;
    const double2 *C = reinterpret_cast<const double2 *>(coef);
    const size_t spin_stride = (size_t)nb * nsp;  // complex elements
    const double *Xp = XT + pt0 + li;

    acc_t acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = acc_t{0, 0, 0, 0};
    auto mfma = [](double a, double b, acc_t c) -> acc_t {
        if constexpr (__is_same(T, double))
            return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
    };

    // K-steps of this wave: mu groups mu_lo + 4 wave + 16 j.  They are
    // fetched in batches of BK into registers; batch b + 1 is requested before
    // the MFMAs of batch b are issued, so its loads overlap BK x 4 MFMAs.
    // BK = 2 keeps the FP64 kernel at four waves per SIMD, so every block of
    // a 128-pair launch is resident at once (measured faster than BK = 4 or 8,
    // whose larger stages cost occupancy).
    constexpr int BK = 2;
    struct Stage {
        double x[BK];
        double2 ca[BK], cb[BK];
    };
    auto fetch = [&](int mu_first, Stage &st) {
        for (int j = 0; j < BK; ++j) {
            const int mu = min(mu_first + 16 * j + lk, mu_hi - 1);
            st.x[j] = Xp[(size_t)mu * E];
            st.ca[j] = C[(size_t)mu * nsp + kc];
            st.cb[j] = C[spin_stride + (size_t)mu * nsp + kc];
        }
    };
    auto consume = [&](int mu_first, const Stage &st) {
        for (int j = 0; j < BK; ++j) {
            const bool ok = mu_first + 16 * j + lk < mu_hi;
            const double xv = ok ? st.x[j] : 0.0;
            const bool okc = ok && k_ok;
            acc[0] = mfma(okc ? st.ca[j].x : 0.0, xv, acc[0]);
            acc[1] = mfma(okc ? st.ca[j].y : 0.0, xv, acc[1]);
            acc[2] = mfma(okc ? st.cb[j].x : 0.0, xv, acc[2]);
            acc[3] = mfma(okc ? st.cb[j].y : 0.0, xv, acc[3]);
        }
    };
    const int mu_w = mu_lo + 4 * wave;
    const int n_batches = (mu_hi - mu_w + 16 * BK - 1) / (16 * BK);
    // Two register stages used alternately (no copies between them);
    // sched_barrier(0) keeps the scheduler from sinking a batch's loads below
    // the MFMAs they are meant to overlap.
    // The loop body is branch-free (fetches past the end read clamped, valid
    // addresses and are masked when consumed), so the waits the compiler
    // inserts before each consume cover only the older stage's loads.
    Stage sa, sb;
    fetch(mu_w, sa);
    for (int b = 0; b < n_batches; b += 2) {
        const int mu_b = mu_w + 16 * BK * b;
        fetch(mu_b + 16 * BK, sb);
        __builtin_amdgcn_sched_barrier(0);
        consume(mu_b, sa);
        __builtin_amdgcn_sched_barrier(0);
        fetch(mu_b + 32 * BK, sa);
        __builtin_amdgcn_sched_barrier(0);
        consume(mu_b + 16 * BK, sb);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (wave > 0)
        for (int q = 0; q < 4; ++q) red[wave - 1][q][lane] = acc[q];
    __syncthreads();
    if (wave != 0) return;
    for (int w = 0; w < 3; ++w)
        for (int q = 0; q < 4; ++q) acc[q] += red[w][q][lane];
    const int pt = pt0 + li;
    typedef T pair_t __attribute__((ext_vector_type(2)));
    pair_t *out = reinterpret_cast<pair_t *>(psi_out);
    for (int v = 0; v < 4; ++v) {
        const int kk = __is_same(T, double) ? k0 + 4 * v + lk : k0 + 4 * lk + v;  // result row of element v
        if (kk >= nsp) continue;
        out[(size_t)kk * R + 4 * pt + 2 * set] = pair_t{acc[0][v], acc[1][v]};      // alpha
        out[(size_t)kk * R + 4 * pt + 2 * set + 1] = pair_t{acc[2][v], acc[3][v]};  // beta
    }
}


// Spinor values on FP64 / FP32 MFMA (Eq. (C)):
//   psi[k][4 pt + 2 set + s] = sum_{mu in set} C[s][mu][k] chi_mu(r_pt)
// One block: KS spinors x PTS points of one primitive set (L or S), both
// spins, real and imaginary parts.  As a real GEMM D[r][pt] = sum_mu
// A[r][mu] B[mu][pt]: B = XT, A rows r = (spinor k, q = 2 s + ri).  Inside
// each 16-row MFMA tile the rows are ordered so that a lane's four result
// elements are the four q of one spinor: r = 4 q + kk for the FP64 MFMA
// (element v at row 4 v + l / 16) and r = 4 kk + q for the FP32 MFMA
// (element v at row 4 (l / 16) + v).  Operand layout of v_mfma_*_16x16x4:
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] (checked on gfx950).
// K chunks of 16 primitives go through LDS (double-buffered; registers
// prefetch the next chunk): As[mu][k][s][ri] and Bs[mu][pt], each mu row
// padded by 128 B so that 16 lanes read 128 contiguous bytes and the four
// K-groups of a wave fall 128 B apart modulo the 256-byte bank row.
// Work items (spinor tile, point tile, set) are dealt to the XCDs in
// contiguous ranges of tile pairs (spinor_set_item: block b runs on XCD
// b % 8), so the point tiles sharing a coefficient tile read it through one
// L2; within a range the longer small-component items go first.
typedef double d2v __attribute__((ext_vector_type(2)));

template <typename T, int KS, int PTS>
__global__ __launch_bounds__(256) void spinor_tile_kernel(const double *__restrict__ XT,
                                                          const double *__restrict__ coef, int E, int nb, int nL,
                                                          int nsp, int R, int n_kt, int n_pt,
                                                          void *__restrict__ psi_out) {
    constexpr int KC = 16;                 // primitives per chunk
    constexpr int AROW = 4 * KS + 16;      // doubles per mu row of As
    constexpr int BROW = PTS + 16;         // doubles per mu row of Bs
    constexpr int WR = KS / 8;             // 16-row MFMA tiles per wave (a wave owns 2 KS rows)
    constexpr int WP = PTS / 32;           // 16-point MFMA tiles per wave
    constexpr int NAU = KC * 2 * KS;       // 16-byte A units per chunk: (mu, s, k) complex
    constexpr int NBU = KC * PTS / 2;      // 16-byte B units per chunk: (mu, two points)
    constexpr int PA = (NAU + 255) / 256, PB = (NBU + 255) / 256;
    static_assert(KS % 8 == 0 && PTS % 32 == 0, "tile shape");
    typedef T acc_t __attribute__((ext_vector_type(4)));
    __shared__ __align__(16) double As[2][KC * AROW];
    __shared__ __align__(16) double Bs[2][KC * BROW];

    int set, rest;
    if (!spinor_set_item(n_kt * n_pt, set, rest)) return;
    const int k0 = (rest / n_pt) * KS, pt0 = (rest % n_pt) * PTS;
    const int mu_lo = set ? nL : 0, mu_hi = set ? nb : nL;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;

    d2v ra[PA], rb[PB];
    // Loads are branch-free: indices past the end read the last valid element.
    // Primitives past the set's end are zeroed (they must not contribute) when
    // the chunk is staged, so the loads' wait falls at the LDS store, after the
    // current chunk's MFMAs (a select at load time made the compiler wait for
    // the whole prefetch before them).
    auto gload = [&](int mu0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PA; ++j) {
            const int u = min(tid + 256 * j, NAU - 1);
            const int ml = u / (2 * KS), sp = (u / KS) & 1, k = u % KS;
            ra[j] = *reinterpret_cast<const d2v *>(
                coef + 2 * (((size_t)sp * nb + min(mu0 + ml, mu_hi - 1)) * nsp + min(k0 + k, nsp - 1)));
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int u = min(tid + 256 * j, NBU - 1);
            const int ml = u / (PTS / 2), p2 = u % (PTS / 2);
            rb[j] = *reinterpret_cast<const d2v *>(XT + (size_t)min(mu0 + ml, mu_hi - 1) * E +
                                                   min(pt0 + 2 * p2, E - 2));
        }
    };
    auto lstore = [&](int buf, int mu0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PA; ++j) {
            const int u = min(tid + 256 * j, NAU - 1);
            const int ml = u / (2 * KS), sp = (u / KS) & 1, k = u % KS;
            *reinterpret_cast<d2v *>(&As[buf][ml * AROW + 4 * k + 2 * sp]) =
                mu0 + ml < mu_hi ? ra[j] : d2v{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int u = min(tid + 256 * j, NBU - 1);
            const int ml = u / (PTS / 2), p2 = u % (PTS / 2);
            *reinterpret_cast<d2v *>(&Bs[buf][ml * BROW + 2 * p2]) = mu0 + ml < mu_hi ? rb[j] : d2v{0.0, 0.0};
        }
    };
    acc_t acc[WR][WP];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WP; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    // A row of this lane inside a 16-row tile: (q, kk) per the MFMA's result layout
    constexpr bool F64 = __is_same(T, double);
    const int q = F64 ? li >> 2 : li & 3, kk = F64 ? li & 3 : li >> 2;
    const int a_off = lk * AROW + 4 * (4 * WR * wr + kk) + q;  // + 16 i (next spinor group) + 4 ks AROW
    const int b_off = lk * BROW + (PTS / 2) * wc + li;        // + 16 j + 4 ks BROW

    const int n_chunks = (mu_hi - mu_lo + KC - 1) / KC;
    gload(mu_lo);
    lstore(0, mu_lo);
    __syncthreads();
    for (int c = 0; c < n_chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < n_chunks) gload(mu_lo + KC * (c + 1));
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            T a[WR], bv[WP];
#pragma unroll
            for (int i = 0; i < WR; ++i) a[i] = (T)As[buf][a_off + 16 * i + 4 * ks * AROW];
#pragma unroll
            for (int j = 0; j < WP; ++j) bv[j] = (T)Bs[buf][b_off + 16 * j + 4 * ks * BROW];
#pragma unroll
            for (int i = 0; i < WR; ++i)
#pragma unroll
                for (int j = 0; j < WP; ++j) {
                    if constexpr (F64)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv[j], acc[i][j], 0, 0, 0);
                }
        }
        if (c + 1 < n_chunks) lstore(buf ^ 1, mu_lo + KC * (c + 1));
        __syncthreads();
    }

    // element v of acc[i][j] = part q = v of spinor k0 + 4 (WR wr + i) + lk at point pt0 + (PTS / 2) wc + 16 j + li
    typedef T pair_t __attribute__((ext_vector_type(2)));
    pair_t *out = reinterpret_cast<pair_t *>(psi_out);
#pragma unroll
    for (int i = 0; i < WR; ++i) {
        const int k = k0 + 4 * (WR * wr + i) + lk;
        if (k >= nsp) continue;
#pragma unroll
        for (int j = 0; j < WP; ++j) {
            const int pt = pt0 + (PTS / 2) * wc + 16 * j + li;
            if (pt >= E) continue;
            pair_t *o = out + (size_t)k * R + 4 * pt + 2 * set;
            o[0] = pair_t{acc[i][j][0], acc[i][j][1]};  // alpha
            o[1] = pair_t{acc[i][j][2], acc[i][j][3]};  // beta
        }
    }
}

template <typename T, int KS, int PTS>
hipError_t launch_spinor_tile(const mcmp2_ctx *c) {
    const int n_kt = (c->nsp + KS - 1) / KS, n_pt = (c->E + PTS - 1) / PTS;
    spinor_tile_kernel<T, KS, PTS><<<16 * ((n_kt * n_pt + 7) / 8), 256, 0, c->stream>>>(
        c->XT, c->coef, c->E, c->nb, c->nL, c->nsp, c->R, n_kt, n_pt, c->psi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spinor_typed(const mcmp2_ctx *c) {
    auto items = [&](int ks, int pts) { return 2 * ((c->nsp + ks - 1) / ks) * ((c->E + pts - 1) / pts); };
    if (items(16, 64) >= 4 * c->n_cu) return launch_spinor_tile<T, 16, 64>(c);
    if (items(32, 128) >= c->n_cu) return launch_spinor_tile<T, 32, 128>(c);
    if (items(16, 64) >= c->n_cu) return launch_spinor_tile<T, 16, 64>(c);
    // latency-bound sizes: 16 x 16 tiles, K split over the block's waves, no LDS staging
    dim3 grid((c->nsp + 15) / 16, c->E / 16, 2);
    spinor_gemm_kernel<T><<<grid, 256, 0, c->stream>>>(c->XT, c->coef, c->E, c->nb, c->nL, c->nsp, c->R, c->psi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_prep(const mcmp2_ctx *c, const double *walkers, const double *tau, int n_tau) {
    // the tiled BF16 / FP16 spinor GEMM reads only the BF16 basis values
    if ((c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16) && spinor_lp_tiled(c))
        return launch_step_prep_lp(c, walkers, tau, n_tau);
    const int n_pts = 2 * c->m;
    dim3 grid((n_pts + 127) / 128, c->nb + 1);
    step_prep_kernel<<<grid, 128, 0, c->stream>>>(
        walkers, n_pts, c->E, c->nb, reinterpret_cast<const double4 *>(c->pgeo),
        reinterpret_cast<const double2 *>(c->pnl), c->XT, c->m, c->nuc, c->gpar, c->n_nuc, c->Ng, c->hinv, c->rhat, tau,
        c->eps,
        n_tau, c->nsp, c->no, c->lambda, c->scale, c->wtau);
    return hipGetLastError();
}

// BF16 / FP16 modes: the split-BF16 128x128-tile GEMM when it has a tile per
// two CUs; below that it is latency-bound, and the FP32 path (FP32 MFMA on
// operands rounded from FP64, the more accurate of the two) writes the same
// float2 psi in less time.
hipError_t launch_spinor_gemm(const mcmp2_ctx *c) {
    if (c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16) {
        if (spinor_lp_tiled(c)) return launch_spinor_lp(c);
        const hipError_t e = launch_x_lp(c, false);  // XTb of the coefficient gradient, if requested
        if (e != hipSuccess) return e;
        return launch_spinor_typed<float>(c);
    }
    return c->precision == MCMP2_FP64 ? launch_spinor_typed<double>(c) : launch_spinor_typed<float>(c);
}
