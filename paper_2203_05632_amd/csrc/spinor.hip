// Spinor values at the walker positions (Sec. II, Eq. (C) of the paper):
//   phi_k^{L s}(r) = sum_{mu in L} C[s][mu][k] chi_mu(r),
//   phi_k^{S s}(r) = sum_{mu in S} C[s][mu][k] chi_mu(r),
// for the 2m electron positions of a step.  chi_mu is a Cartesian primitive
// N (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-zeta |r-A|^2).
//
// Two kernels:
//   basis_values  -- XT[mu][pt] = chi_mu(r_pt), FP64, point index fastest;
//   spinor_gemm   -- psi[k][4 pt + c] (complex), a real x complex GEMM on
//                    FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// psi is stored spinor-major with the row index r = 4 pt + c = 8 p + 4 e + c
// (pair p, electron e, component c in L alpha, L beta, S alpha, S beta)
// fastest, so that a 16-row slice for one spinor is 256 contiguous bytes:
// this is the operand layout the Green's-function kernel streams.
#include "internal.hpp"

namespace {

__global__ void basis_values_kernel(const double *__restrict__ walkers, int n_pts, int E, int nb,
                                    const double *__restrict__ pxyz, const double *__restrict__ pexp,
                                    const double *__restrict__ pnorm, const int *__restrict__ plxyz,
                                    double *__restrict__ XT) {
    int pt = blockIdx.x * blockDim.x + threadIdx.x;
    int mu = blockIdx.y;
    if (pt >= n_pts) return;
    double dx = walkers[3 * pt] - pxyz[3 * mu];
    double dy = walkers[3 * pt + 1] - pxyz[3 * mu + 1];
    double dz = walkers[3 * pt + 2] - pxyz[3 * mu + 2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double poly = 1.0;
    for (int i = 0; i < plxyz[3 * mu]; ++i) poly *= dx;
    for (int i = 0; i < plxyz[3 * mu + 1]; ++i) poly *= dy;
    for (int i = 0; i < plxyz[3 * mu + 2]; ++i) poly *= dz;
    XT[(size_t)mu * E + pt] = pnorm[mu] * poly * exp(-pexp[mu] * r2);
}

// One wave computes a 16 (spinor k) x 16 (point) tile of one component set
// (blockIdx.z: 0 = L, 1 = S) for both spins, re and im: four 16x16 FP64
// accumulators.  MFMA operand layout (16x16x4 f64): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the result D[4 v + l / 16][l % 16]
// sits in element v of the lane's accumulator (checked on gfx950).
__global__ __launch_bounds__(256) void spinor_gemm_kernel(const double *__restrict__ XT,
                                                          const double *__restrict__ coef, int E, int nb,
                                                          int nL, int nsp, int R, double *__restrict__ psi) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int set = blockIdx.z;
    const int k0 = blockIdx.x * 16;
    const int pt0 = (blockIdx.y * 4 + wave) * 16;
    if (pt0 >= E) return;
    const int mu_lo = set == 0 ? 0 : nL;
    const int mu_hi = set == 0 ? nL : nb;
    const int li = lane & 15, lk = lane >> 4;
    const int k = k0 + li;

    d4v acc[2][2];
    for (int s = 0; s < 2; ++s)
        for (int q = 0; q < 2; ++q) acc[s][q] = d4v{0.0, 0.0, 0.0, 0.0};

    const size_t spin_stride = (size_t)nb * nsp;  // complex elements
    for (int mu0 = mu_lo; mu0 < mu_hi; mu0 += 4) {
        int mu = mu0 + lk;
        double x = 0.0, car = 0.0, cai = 0.0, cbr = 0.0, cbi = 0.0;
        if (mu < mu_hi) {
            x = XT[(size_t)mu * E + pt0 + li];
            if (k < nsp) {
                const double2 ca = reinterpret_cast<const double2 *>(coef)[(size_t)mu * nsp + k];
                const double2 cb = reinterpret_cast<const double2 *>(coef)[spin_stride + (size_t)mu * nsp + k];
                car = ca.x;
                cai = ca.y;
                cbr = cb.x;
                cbi = cb.y;
            }
        }
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(car, x, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(cai, x, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(cbr, x, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(cbi, x, acc[1][1], 0, 0, 0);
    }
    const int pt = pt0 + li;
    for (int v = 0; v < 4; ++v) {
        const int kk = k0 + 4 * v + lk;
        if (kk >= nsp) continue;
        for (int s = 0; s < 2; ++s) {
            const int c = 2 * set + s;
            double2 val = {acc[s][0][v], acc[s][1][v]};
            reinterpret_cast<double2 *>(psi)[(size_t)kk * R + 4 * pt + c] = val;
        }
    }
}

}  // namespace

hipError_t launch_basis_values(const mcmp2_ctx *c, const double *walkers) {
    int n_pts = 2 * c->m;
    dim3 grid((n_pts + 127) / 128, c->nb);
    basis_values_kernel<<<grid, 128, 0, c->stream>>>(walkers, n_pts, c->E, c->nb, c->pxyz, c->pexp, c->pnorm,
                                                     c->plxyz, c->XT);
    return hipGetLastError();
}

hipError_t launch_spinor_gemm(const mcmp2_ctx *c) {
    // E is a multiple of 16; four point tiles per 256-thread block.
    int pt_tiles = c->E / 16;
    dim3 grid((c->nsp + 15) / 16, (pt_tiles + 3) / 4, 2);
    spinor_gemm_kernel<<<grid, 256, 0, c->stream>>>(c->XT, c->coef, c->E, c->nb, c->nL, c->nsp, c->R, c->psi);
    return hipGetLastError();
}
