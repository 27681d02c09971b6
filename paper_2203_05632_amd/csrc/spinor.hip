// Spinor values at the walker positions (Sec. II, Eq. (C) of the paper):
//   phi_k^{L s}(r) = sum_{mu in L} C[s][mu][k] chi_mu(r),
//   phi_k^{S s}(r) = sum_{mu in S} C[s][mu][k] chi_mu(r),
// for the 2m electron positions of a step, where chi_mu is a Cartesian
// primitive N (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-zeta |r-A|^2).
//
// Two kernels:
//   step_prep    -- XT[mu][pt] = chi_mu(r_pt) (FP64, point index fastest),
//                   plus the per-step scalars the Green's-function kernel
//                   needs: N_g / (g(r1p) g(r2p)) per walker, the tau scalings
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

// chi_mu(r) for the packed primitive record (A, zeta) + (N, lx | ly << 8 | lz << 16)
__device__ inline double basis_value(const double4 &geo, const double2 &nl, double x, double y, double z) {
    const double dx = x - geo.x, dy = y - geo.y, dz = z - geo.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const int l = (int)__double_as_longlong(nl.y);  // packed powers, bit pattern stored in a double
    double poly = 1.0;
    for (int i = 0; i < (l & 0xff); ++i) poly *= dx;
    for (int i = 0; i < ((l >> 8) & 0xff); ++i) poly *= dy;
    for (int i = 0; i < ((l >> 16) & 0xff); ++i) poly *= dz;
    return nl.x * poly * exp(-geo.w * r2);
}

// grid (ceil(n_pts / 128), nb + 1): rows y < nb evaluate basis function y at
// every point; row y == nb runs a grid-stride loop over the walker factors,
// the tau scalings and the tau weights.
__global__ __launch_bounds__(128) void step_prep_kernel(
    const double *__restrict__ walkers, int n_pts, int E, int nb, const double4 *__restrict__ pgeo,
    const double2 *__restrict__ pnl, double *__restrict__ XT, int m, const double *__restrict__ nuc,
    const double *__restrict__ gpar, int n_nuc, double Ng, double *__restrict__ hinv, const double *__restrict__ tau,
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
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) {
        if (i < m) {
            const double *r = walkers + 6 * i;
            const double g1 = g_value(r[0], r[1], r[2], nuc, gpar, n_nuc);
            const double g2 = g_value(r[3], r[4], r[5], nuc, gpar, n_nuc);
            hinv[i] = Ng / (g1 * g2);
        } else if (i < m + n_tau * nsp) {
            const int j = i - m, t = j / nsp, k = j - t * nsp;
            const double tv = tau[t];
            scale[j] = k < no ? exp(eps[k] * tv) : exp(-eps[k] * tv);
        } else {
            const int t = i - m - n_tau * nsp;
            wtau[t] = lambda * exp(-lambda * tau[t]);
        }
    }
}

// One block computes a 16 (spinor k) x 16 (point) tile of one component set
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
    constexpr int BK = 8;
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

}  // namespace

hipError_t launch_step_prep(const mcmp2_ctx *c, const double *walkers, const double *tau, int n_tau) {
    const int n_pts = 2 * c->m;
    dim3 grid((n_pts + 127) / 128, c->nb + 1);
    step_prep_kernel<<<grid, 128, 0, c->stream>>>(
        walkers, n_pts, c->E, c->nb, reinterpret_cast<const double4 *>(c->pgeo),
        reinterpret_cast<const double2 *>(c->pnl), c->XT, c->m, c->nuc, c->gpar, c->n_nuc, c->Ng, c->hinv, tau, c->eps,
        n_tau, c->nsp, c->no, c->lambda, c->scale, c->wtau);
    return hipGetLastError();
}

hipError_t launch_spinor_gemm(const mcmp2_ctx *c) {
    if (c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16) return launch_spinor_lp(c);
    dim3 grid((c->nsp + 15) / 16, c->E / 16, 2);
    if (c->precision == MCMP2_FP64)
        spinor_gemm_kernel<double><<<grid, 256, 0, c->stream>>>(c->XT, c->coef, c->E, c->nb, c->nL, c->nsp, c->R,
                                                                c->psi);
    else
        spinor_gemm_kernel<float><<<grid, 256, 0, c->stream>>>(c->XT, c->coef, c->E, c->nb, c->nL, c->nsp, c->R,
                                                               c->psi);
    return hipGetLastError();
}
