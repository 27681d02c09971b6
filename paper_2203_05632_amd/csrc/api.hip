// C ABI of libmcmp2 (declared in include/mcmp2.h): context set-up, the
// per-step driver of the hot path and the sampler entry points.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

namespace {
thread_local char g_err[512] = "";

// Two-centre Coulomb integral of unnormalised s Gaussians:
// int int exp(-a|r1-A|^2) exp(-b|r2-B|^2) / r12 = 2 pi^(5/2)/(a b sqrt(a+b)) F0(ab/(a+b) R^2).
double coulomb_ss(double a, double b, double R2) {
    const double T = a * b / (a + b) * R2;
    const double F0 = T < 1e-14 ? 1.0 - T / 3.0 : 0.5 * std::sqrt(M_PI / T) * std::erf(std::sqrt(T));
    return 2.0 * std::pow(M_PI, 2.5) / (a * b * std::sqrt(a + b)) * F0;
}

double s_norm(double z) { return std::pow(2.0 * z / M_PI, 0.75); }

template <class T>
int dalloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        set_error("hipMalloc of %zu bytes failed", n * sizeof(T));
        return MCMP2_ENOMEM;
    }
    return MCMP2_OK;
}

void profiler_release(Profiler &p);
void free_ctx(mcmp2_ctx *c) {
    profiler_release(c->prof);
    void *bufs[] = {c->nuc, c->gpar, c->pgeo, c->pnl, c->coef, c->eps, c->hinv, c->rhat, c->psi,
                    c->scale, c->wtau, c->tiles, c->work, c->partial, c->XT,
                    c->Hm, c->Hp, c->psibar, c->eps_part, c->U, c->Vt, c->tiles16,
                    c->Cb, c->Xb, c->XTb, c->PBb, c->gstage};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete c;
}
}  // namespace

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return MCMP2_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return MCMP2_EDEVICE;
}

namespace {
// Launch through `fn`, bracketed by an event pair when kernel `kid` is being timed.
// The stage's slot is taken before fn runs, so dispatch-level pairs recorded
// inside fn (prof_begin / prof_end) take the slots after it.
template <class F>
int timed(mcmp2_ctx *c, int kid, const char *what, F fn) {
    const int slot = prof_begin(c, kid);
    int rc = check_hip(fn(), what);
    if (rc != MCMP2_OK) return rc;
    return check_hip(prof_end(c, slot, kid), "hipEventRecord");
}

void profiler_release(Profiler &p) {
    if (p.ev) {
        for (int i = 0; i < 2 * p.capacity; ++i)
            if (p.ev[i]) (void)hipEventDestroy(p.ev[i]);
    }
    delete[] p.ev;
    delete[] p.kid;
    p = Profiler();
}
}  // namespace

#define TRY(x)                     \
    do {                           \
        int rc_ = (x);             \
        if (rc_ != MCMP2_OK) {     \
            free_ctx(c);           \
            return rc_;            \
        }                          \
    } while (0)

extern "C" const char *mcmp2_last_error(void) { return g_err; }

int check_setup(const mcmp2_basis *basis, const double *coeffs, const double *eps, int n_occ, int n_vir,
                int m_pairs, int n_tau_max, int precision, double *lambda_out) {
    if (!basis || !coeffs || !eps || !basis->nuc_xyz || !basis->wfn || !basis->prim_xyz || !basis->prim_exp ||
        !basis->prim_lxyz || !basis->prim_norm) {
        set_error("null input pointer");
        return MCMP2_EINVAL;
    }
    if (basis->n_nuc < 1 || basis->n_L < 1 || basis->n_S < 0 || n_occ < 1 || n_vir < 1 || m_pairs < 2 ||
        n_tau_max < 1) {
        set_error("sizes out of range: n_nuc=%d n_L=%d n_S=%d n_occ=%d n_vir=%d m=%d n_tau_max=%d", basis->n_nuc,
                  basis->n_L, basis->n_S, n_occ, n_vir, m_pairs, n_tau_max);
        return MCMP2_EINVAL;
    }
    if (precision < MCMP2_FP64 || precision > MCMP2_FP16) {
        set_error("precision %d is not one of MCMP2_FP64, _FP32, _BF16, _FP16", precision);
        return MCMP2_EINVAL;
    }
    const int nb = basis->n_L + basis->n_S;
    for (int i = 0; i < nb; ++i) {
        for (int d = 0; d < 3; ++d) {
            int l = basis->prim_lxyz[3 * i + d];
            if (l < 0 || l > 4) {
                set_error("primitive %d: Cartesian power %d out of range 0..4", i, l);
                return MCMP2_EINVAL;
            }
        }
        if (!(basis->prim_exp[i] > 0.0)) {
            set_error("primitive %d: exponent must be positive", i);
            return MCMP2_EINVAL;
        }
    }
    for (int I = 0; I < basis->n_nuc; ++I)
        if (!(basis->wfn[4 * I + 1] > 0.0) || !(basis->wfn[4 * I + 3] > 0.0)) {
            set_error("nucleus %d: weight-function exponents must be positive", I);
            return MCMP2_EINVAL;
        }
    const int nsp = n_occ + n_vir;
    double homo = eps[0], lumo = eps[n_occ];
    for (int i = 0; i < n_occ; ++i) homo = std::max(homo, eps[i]);
    for (int a = n_occ; a < nsp; ++a) lumo = std::min(lumo, eps[a]);
    const double lambda = 2.0 * (lumo - homo);
    if (!(lambda > 0.0)) {
        set_error("lambda = 2 (eps_LUMO - eps_HOMO) = %g must be positive", lambda);
        return MCMP2_EINVAL;
    }
    *lambda_out = lambda;
    return MCMP2_OK;
}

int setup_ctx(mcmp2_ctx *c, const mcmp2_basis *basis, int n_occ, int n_vir, int m_pairs, int n_tau_max,
              int precision, int want_grad, double lambda, void *hip_stream, std::vector<double> &gpar) {
    if (hipGetDevice(&c->device) != hipSuccess) {
        set_error("no HIP device");
        return MCMP2_EDEVICE;
    }
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        c->n_cu < 1)
        c->n_cu = 256;
    c->stream = (hipStream_t)hip_stream;
    c->n_nuc = basis->n_nuc;
    c->nL = basis->n_L;
    c->nS = basis->n_S;
    c->nb = basis->n_L + basis->n_S;
    c->no = n_occ;
    c->nv = n_vir;
    c->nsp = n_occ + n_vir;
    c->m = m_pairs;
    c->m_pad = (m_pairs + kWalkerPad - 1) / kWalkerPad * kWalkerPad;
    c->E = 2 * c->m_pad;
    c->R = 8 * c->m_pad;
    c->T = c->m_pad / kTileWalkers;
    c->n_tp = c->T * (c->T + 1) / 2;
    c->n_tau_max = n_tau_max;
    c->precision = precision;
    c->want_grad = want_grad;
    c->lambda = lambda;
    // BF16 / FP16 operand layout: K extents (reals) padded to multiples of the
    // K chunk (64) of their Green's-function kernels
    const int kq = 64;
    c->Ko = (2 * n_occ + kq - 1) / kq * kq;
    c->Ktot = c->Ko + (2 * n_vir + kq - 1) / kq * kq;

    // N_g = sum over all pairs of weight-function Gaussians (Sec. III).
    gpar.assign(4 * (size_t)c->n_nuc, 0.0);
    double Ng = 0.0;
    for (int I = 0; I < c->n_nuc; ++I) {
        const double *w = basis->wfn + 4 * I;
        gpar[4 * I] = w[0] * s_norm(w[1]);
        gpar[4 * I + 1] = w[1];
        gpar[4 * I + 2] = w[2] * s_norm(w[3]);
        gpar[4 * I + 3] = w[3];
    }
    for (int I = 0; I < c->n_nuc; ++I)
        for (int ka = 0; ka < 2; ++ka)
            for (int J = 0; J < c->n_nuc; ++J)
                for (int kb = 0; kb < 2; ++kb) {
                    const double *A = basis->nuc_xyz + 3 * I, *B = basis->nuc_xyz + 3 * J;
                    double R2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                                (A[2] - B[2]) * (A[2] - B[2]);
                    Ng += gpar[4 * I + 2 * ka] * gpar[4 * J + 2 * kb] *
                          coulomb_ss(gpar[4 * I + 2 * ka + 1], gpar[4 * J + 2 * kb + 1], R2);
                }
    c->Ng = Ng;
    return MCMP2_OK;
}

void triangle_tiles(int T, std::vector<int> &tiles) {
    tiles.clear();
    tiles.reserve((size_t)T * (T + 1));
    for (int P = 0; P < T; ++P)
        for (int Q = P; Q < T; ++Q) {
            tiles.push_back(P);
            tiles.push_back(Q);
        }
}

double green_tile_bytes(const mcmp2_ctx *c) {
    // bytes of one block tile's operand rows: 8 kTileWalkers rows of all spinors
    const double row_bytes = c->precision == MCMP2_FP64 ? 16.0 * c->nsp
                             : c->precision == MCMP2_FP32 ? 8.0 * c->nsp
                                                          : 2.0 * c->Ktot;
    return 8.0 * kTileWalkers * row_bytes;
}

void pack_basis(const mcmp2_basis *basis, std::vector<double> &geo, std::vector<double> &nl) {
    const int nb = basis->n_L + basis->n_S;
    geo.assign(4 * (size_t)nb, 0.0);
    nl.assign(2 * (size_t)nb, 0.0);
    for (int i = 0; i < nb; ++i) {
        for (int d = 0; d < 3; ++d) geo[4 * i + d] = basis->prim_xyz[3 * i + d];
        geo[4 * i + 3] = basis->prim_exp[i];
        nl[2 * i] = basis->prim_norm[i];
        const int64_t packed = (int64_t)basis->prim_lxyz[3 * i] | ((int64_t)basis->prim_lxyz[3 * i + 1] << 8) |
                               ((int64_t)basis->prim_lxyz[3 * i + 2] << 16);
        std::memcpy(&nl[2 * i + 1], &packed, sizeof(double));
    }
}

extern "C" int mcmp2_init(const mcmp2_basis *basis, const double *coeffs, const double *eps, int32_t n_occ,
                          int32_t n_vir, int32_t m_pairs, int32_t n_tau_max, int32_t precision, int32_t want_grad,
                          void *hip_stream, mcmp2_ctx **out) {
    g_err[0] = '\0';
    if (!out) {
        set_error("out is NULL");
        return MCMP2_EINVAL;
    }
    *out = nullptr;
    double lambda = 0.0;
    int rc0 = check_setup(basis, coeffs, eps, n_occ, n_vir, m_pairs, n_tau_max, precision, &lambda);
    if (rc0 != MCMP2_OK) return rc0;
    const int nb = basis->n_L + basis->n_S;
    const int nsp = n_occ + n_vir;

    mcmp2_ctx *c = new (std::nothrow) mcmp2_ctx();
    if (!c) {
        set_error("host allocation failed");
        return MCMP2_ENOMEM;
    }
    std::vector<double> gpar;
    rc0 = setup_ctx(c, basis, n_occ, n_vir, m_pairs, n_tau_max, precision, want_grad, lambda, hip_stream, gpar);
    if (rc0 != MCMP2_OK) {
        delete c;
        return rc0;
    }
    const size_t op_bytes = 2;
    std::vector<int> tiles;
    triangle_tiles(c->T, tiles);

    TRY(dalloc(&c->nuc, 3 * (size_t)c->n_nuc));
    TRY(dalloc(&c->gpar, 4 * (size_t)c->n_nuc));
    TRY(dalloc(&c->pgeo, 4 * (size_t)nb));
    TRY(dalloc(&c->pnl, 2 * (size_t)nb));
    TRY(dalloc(&c->coef, 2 * 2 * (size_t)nb * nsp));
    TRY(dalloc(&c->eps, (size_t)nsp));
    TRY(dalloc(&c->hinv, (size_t)c->m_pad));
    TRY(dalloc(&c->rhat, 4 * (size_t)c->m_pad));
    TRY(dalloc(&c->psi, 2 * (size_t)nsp * c->R));  // double2 (FP64) or float2 (low precision)
    if (precision == MCMP2_BF16 || precision == MCMP2_FP16) {
        unsigned char *u = nullptr;
        const size_t ub = op_bytes * (size_t)n_tau_max * c->R * c->Ktot;
        TRY(dalloc(&u, ub));
        c->U = u;
        TRY(check_hip(hipMemset(c->U, 0, ub), "hipMemset"));  // K padding stays zero
    }
    if (precision == MCMP2_BF16 || precision == MCMP2_FP16) {
        auto r64 = [](int v) { return (v + 63) / 64 * 64; };
        c->nLp = r64(c->nL);
        c->nbp = c->nLp + r64(c->nS);
        c->Ep = r64(c->E);
        auto zalloc = [&](void **p, size_t bytes) {
            unsigned char *b = nullptr;
            int rc = dalloc(&b, bytes);
            *p = b;
            if (rc == MCMP2_OK) rc = check_hip(hipMemset(b, 0, bytes), "hipMemset");
            return rc;
        };
        TRY(zalloc(&c->Cb, 2 * (size_t)4 * nsp * 3 * c->nbp));  // BF16, split rows of 3 nbp
        TRY(zalloc(&c->Xb, 2 * (size_t)c->E * 3 * c->nbp));
        if (want_grad) {
            TRY(zalloc(&c->XTb, 2 * (size_t)nb * c->Ep));
            TRY(zalloc(&c->PBb, 2 * (size_t)2 * 4 * nsp * c->Ep));
        }
    }
    TRY(dalloc(&c->scale, (size_t)n_tau_max * nsp));
    TRY(dalloc(&c->wtau, (size_t)n_tau_max));
    std::vector<int> work;
    build_green_work(c->T, green_tile_bytes(c), work);
    c->n_slots = 4 * (int)work.size();
    TRY(dalloc(&c->tiles, 2 * (size_t)c->n_tp));
    TRY(dalloc(&c->work, work.size()));
    std::vector<int> tiles16;
    if (precision == MCMP2_BF16 || precision == MCMP2_FP16) {
        c->T16 = (c->m_pad + 15) / 16;
        build_big_tiles(c->T16, tiles16);
        c->n_tp16 = (int)tiles16.size() / 2;
        TRY(dalloc(&c->tiles16, tiles16.size()));
    }
    TRY(dalloc(&c->partial, (size_t)n_tau_max * std::max(c->n_slots, 8 * c->n_tp16) * 2));
    TRY(dalloc(&c->XT, (size_t)nb * c->E));
    if (want_grad) {
        // adjoint blocks: FP64 complex (FP64, FP32 modes) or packed BF16 pairs (BF16, FP16 modes)
        const bool h16 = precision == MCMP2_BF16 || precision == MCMP2_FP16;
        const size_t hbytes = (h16 ? 4 : 16) * (size_t)n_tau_max * c->R * c->R;
        unsigned char *hm = nullptr, *hp = nullptr;
        TRY(dalloc(&hm, hbytes));
        c->Hm = reinterpret_cast<double *>(hm);
        TRY(dalloc(&hp, hbytes));
        c->Hp = reinterpret_cast<double *>(hp);
        if (!h16) TRY(dalloc(&c->psibar, 2 * (size_t)nsp * c->R));  // the 16-bit modes write PBb instead
        TRY(dalloc(&c->eps_part, (size_t)(c->R / 32) * nsp));
        if (h16) TRY(dalloc(&c->Vt, (size_t)n_tau_max * nsp * c->R));
        if (h16 && !coef_grad_lp_fused(c)) TRY(dalloc(&c->gstage, (size_t)((nsp + 1) & ~1) + 4 * (size_t)nb * nsp));
        // blocks that are never written (p = q, padding walkers) must read as zero
        TRY(check_hip(hipMemset(c->Hm, 0, hbytes), "hipMemset"));
        TRY(check_hip(hipMemset(c->Hp, 0, hbytes), "hipMemset"));
    }

    auto up = [&](void *dst, const void *src, size_t bytes) {
        return check_hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
    };
    TRY(up(c->nuc, basis->nuc_xyz, 3 * sizeof(double) * c->n_nuc));
    TRY(up(c->gpar, gpar.data(), gpar.size() * sizeof(double)));
    // packed primitive records: (A, zeta) and (N, powers as int64 bits)
    std::vector<double> geo, nl;
    pack_basis(basis, geo, nl);
    TRY(up(c->pgeo, geo.data(), geo.size() * sizeof(double)));
    TRY(up(c->pnl, nl.data(), nl.size() * sizeof(double)));
    TRY(up(c->coef, coeffs, 2 * 2 * sizeof(double) * (size_t)nb * nsp));
    TRY(up(c->eps, eps, sizeof(double) * nsp));
    if (c->Cb) TRY(check_hip(launch_coef_lp(c), "coef_lp"));
    TRY(up(c->tiles, tiles.data(), tiles.size() * sizeof(int)));
    TRY(up(c->work, work.data(), work.size() * sizeof(int)));
    if (c->n_tp16) TRY(up(c->tiles16, tiles16.data(), tiles16.size() * sizeof(int)));
    // padding rows / points stay zero for the lifetime of the context
    TRY(check_hip(hipMemset(c->XT, 0, sizeof(double) * (size_t)nb * c->E), "hipMemset"));
    TRY(check_hip(hipMemset(c->psi, 0, 2 * sizeof(double) * (size_t)nsp * c->R), "hipMemset"));
    TRY(check_hip(hipMemset(c->hinv, 0, sizeof(double) * c->m_pad), "hipMemset"));
    TRY(check_hip(hipMemset(c->rhat, 0, 4 * sizeof(double) * c->m_pad), "hipMemset"));
    TRY(check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize"));
    *out = c;
    return MCMP2_OK;
}

// One step (Eq. redundant) with the gradients, if any, going to geps / gcoef.
static int run_step(mcmp2_ctx *c, const double *walkers, const double *tau, int32_t n_tau, double *e2_out,
                    double *value, grad_out geps, grad_out gcoef) {
    if (!c || !walkers || !tau || !e2_out) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    if (n_tau < 1 || n_tau > c->n_tau_max) {
        set_error("n_tau=%d outside 1..%d", n_tau, c->n_tau_max);
        return MCMP2_EINVAL;
    }
    const bool grad = geps.any() || gcoef.any();
    if (grad && !c->want_grad) {
        set_error("gradient outputs requested but the context was created with want_grad = 0");
        return MCMP2_ESTATE;
    }
    int rc;
    if ((rc = timed(c, MCMP2_K_STEP_PREP, "step_prep", [&] { return launch_step_prep(c, walkers, tau, n_tau); })) !=
        MCMP2_OK)
        return rc;
    if ((rc = timed(c, MCMP2_K_SPINOR_GEMM, "spinor_gemm", [&] { return launch_spinor_gemm(c); })) != MCMP2_OK)
        return rc;
    if ((rc = timed(c, MCMP2_K_GREEN_CONTRACT, "green_contract", [&] {
             return c->precision == MCMP2_FP64 || c->precision == MCMP2_FP32 ? launch_green_contract(c, n_tau, grad)
                                                                             : launch_green_lp(c, n_tau, grad);
         })) != MCMP2_OK)
        return rc;
    if ((rc = timed(c, MCMP2_K_REDUCE, "reduce", [&] { return launch_reduce(c, n_tau, e2_out); })) != MCMP2_OK)
        return rc;
    if (value && (rc = check_hip(launch_step_value(c, e2_out, n_tau, value), "step_value")) != MCMP2_OK) return rc;
    if (!grad) return MCMP2_OK;
    if ((rc = timed(c, MCMP2_K_GRAD, "adjoint", [&] { return launch_adjoint(c, tau, n_tau, geps); })) != MCMP2_OK)
        return rc;
    if (!gcoef.any()) return MCMP2_OK;
    return timed(c, MCMP2_K_COEF_GRAD, "coef_grad", [&] { return launch_coef_grad(c, gcoef); });
}

extern "C" int mcmp2_step(mcmp2_ctx *c, const double *walkers, const double *tau, int32_t n_tau, double *e2_out,
                          double *value, double *grad_eps, double *grad_coeffs) {
    grad_out geps, gcoef;
    geps.out = grad_eps;
    gcoef.out = grad_coeffs;
    return run_step(c, walkers, tau, n_tau, e2_out, value, geps, gcoef);
}

extern "C" int mcmp2_step_accumulate(mcmp2_ctx *c, const double *walkers, const double *tau, int32_t n_tau,
                                     double *e2_out, double *eps_sum, double *eps_comp, double *coeffs_sum,
                                     double *coeffs_comp) {
    if (!eps_sum || !eps_comp || !coeffs_sum || !coeffs_comp) {
        set_error("null accumulator");
        return MCMP2_EINVAL;
    }
    if (((reinterpret_cast<uintptr_t>(coeffs_sum) | reinterpret_cast<uintptr_t>(coeffs_comp)) & 15) != 0) {
        set_error("coefficient accumulators must be 16-byte aligned (complex FP64)");
        return MCMP2_EINVAL;
    }
    grad_out geps, gcoef;
    if (c && c->gstage) {  // small BF16 / FP16 problems: gradients staged, then added
        geps.out = c->gstage;
        gcoef.out = c->gstage + ((c->nsp + 1) & ~1);
        int rc = run_step(c, walkers, tau, n_tau, e2_out, nullptr, geps, gcoef);
        if (rc != MCMP2_OK) return rc;
        if ((rc = timed(c, MCMP2_K_ACCUMULATE, "accumulate",
                        [&] { return launch_accumulate(c, geps.out, eps_sum, eps_comp, c->nsp); })) != MCMP2_OK)
            return rc;
        return timed(c, MCMP2_K_ACCUMULATE, "accumulate",
                     [&] { return launch_accumulate(c, gcoef.out, coeffs_sum, coeffs_comp, 4 * (int64_t)c->nb * c->nsp); });
    }
    geps.sum = eps_sum;
    geps.comp = eps_comp;
    gcoef.sum = coeffs_sum;
    gcoef.comp = coeffs_comp;
    return run_step(c, walkers, tau, n_tau, e2_out, nullptr, geps, gcoef);
}

extern "C" int mcmp2_set_interaction(mcmp2_ctx *c, int32_t interaction) {
    if (!c) {
        set_error("null context");
        return MCMP2_EINVAL;
    }
    if (interaction < MCMP2_COULOMB || interaction > MCMP2_BREIT) {
        set_error("interaction %d is not one of MCMP2_COULOMB, _GAUNT, _BREIT", interaction);
        return MCMP2_EINVAL;
    }
    c->interaction = interaction;
    return MCMP2_OK;
}

extern "C" int mcmp2_set_coefficients(mcmp2_ctx *c, const double *coeffs, const double *eps) {
    if (!c) {
        set_error("null context");
        return MCMP2_EINVAL;
    }
    int rc = MCMP2_OK;
    if (coeffs)
        rc = check_hip(hipMemcpyAsync(c->coef, coeffs, 2 * 2 * sizeof(double) * (size_t)c->nb * c->nsp,
                                      hipMemcpyDeviceToDevice, c->stream),
                       "hipMemcpyAsync");
    if (rc == MCMP2_OK && coeffs && c->Cb) rc = check_hip(launch_coef_lp(c), "coef_lp");
    if (rc == MCMP2_OK && eps)
        rc = check_hip(hipMemcpyAsync(c->eps, eps, sizeof(double) * c->nsp, hipMemcpyDeviceToDevice, c->stream),
                       "hipMemcpyAsync");
    return rc;
}

extern "C" int mcmp2_pair_weights(mcmp2_ctx *c, const double *walkers, double *w) {
    if (!c || !walkers || !w) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    return check_hip(launch_walker_weights(c, walkers, w, nullptr), "walker_weights");
}

extern "C" int mcmp2_metropolis(mcmp2_ctx *c, double *walkers, double *w, uint64_t key0, uint64_t key1,
                                uint64_t step, double delta, int32_t *n_accepted) {
    if (!c || !walkers || !w) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    if (!(delta > 0.0) || !std::isfinite(delta)) {
        set_error("delta must be finite and positive");
        return MCMP2_EINVAL;
    }
    return timed(c, MCMP2_K_METROPOLIS, "metropolis",
                 [&] { return launch_metropolis(c, walkers, w, key0, key1, step, delta, n_accepted); });
}

extern "C" int mcmp2_advance(mcmp2_ctx *c, double *walkers, double *w, uint64_t key0, uint64_t key1, uint64_t step,
                             double delta, int32_t *n_accepted, int32_t n_tau, double *tau) {
    if (!c || !walkers || !w || !tau) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    if (!(delta > 0.0) || !std::isfinite(delta)) {
        set_error("delta must be finite and positive");
        return MCMP2_EINVAL;
    }
    if (n_tau < 1) {
        set_error("n_tau must be >= 1");
        return MCMP2_EINVAL;
    }
    return timed(c, MCMP2_K_ADVANCE, "advance",
                 [&] { return launch_advance(c, walkers, w, key0, key1, step, delta, n_accepted, n_tau, tau); });
}

extern "C" int mcmp2_sample_tau(mcmp2_ctx *c, uint64_t key0, uint64_t key1, uint64_t step, int32_t n_tau,
                                double *tau) {
    if (!c || !tau) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    if (n_tau < 1) {
        set_error("n_tau must be >= 1");
        return MCMP2_EINVAL;
    }
    return timed(c, MCMP2_K_SAMPLE_TAU, "sample_tau", [&] { return launch_sample_tau(c, key0, key1, step, n_tau, tau); });
}

extern "C" int mcmp2_accumulate(mcmp2_ctx *c, const double *src, double *sum, double *comp, int64_t n) {
    if (!c || n < 0 || (n > 0 && (!src || !sum || !comp))) {
        set_error("null argument or negative n");
        return MCMP2_EINVAL;
    }
    return timed(c, MCMP2_K_ACCUMULATE, "accumulate", [&] { return launch_accumulate(c, src, sum, comp, n); });
}

extern "C" int mcmp2_constants(const mcmp2_ctx *c, double *lambda, double *n_g) {
    if (!c) {
        set_error("null context");
        return MCMP2_EINVAL;
    }
    if (lambda) *lambda = c->lambda;
    if (n_g) *n_g = c->Ng;
    return MCMP2_OK;
}

extern "C" int mcmp2_profile_begin(mcmp2_ctx *c, uint32_t mask, int32_t max_launches) {
    if (!c || max_launches < 1) {
        set_error("null context or max_launches < 1");
        return MCMP2_EINVAL;
    }
    profiler_release(c->prof);
    Profiler &p = c->prof;
    p.ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches]();
    p.kid = new (std::nothrow) int[max_launches];
    if (!p.ev || !p.kid) {
        profiler_release(p);
        set_error("host allocation failed");
        return MCMP2_ENOMEM;
    }
    p.capacity = max_launches;
    for (int i = 0; i < 2 * max_launches; ++i) {
        int rc = check_hip(hipEventCreate(&p.ev[i]), "hipEventCreate");
        if (rc != MCMP2_OK) {
            profiler_release(p);
            return rc;
        }
    }
    p.mask = mask;
    p.used = 0;
    return MCMP2_OK;
}

extern "C" int mcmp2_profile_end(mcmp2_ctx *c, double *total_ms, int64_t *launches) {
    if (!c) {
        set_error("null context");
        return MCMP2_EINVAL;
    }
    Profiler &p = c->prof;
    if (p.capacity == 0) {
        set_error("mcmp2_profile_end without mcmp2_profile_begin");
        return MCMP2_ESTATE;
    }
    int rc = check_hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    double ms[MCMP2_NKERNELS] = {0};
    int64_t n[MCMP2_NKERNELS] = {0};
    for (int i = 0; i < p.used && rc == MCMP2_OK; ++i) {
        if (p.kid[i] < 0) continue;  // a pair whose stop event was not recorded
        float t = 0.f;
        rc = check_hip(hipEventElapsedTime(&t, p.ev[2 * i], p.ev[2 * i + 1]), "hipEventElapsedTime");
        ms[p.kid[i]] += t;
        n[p.kid[i]] += 1;
    }
    profiler_release(p);
    if (rc != MCMP2_OK) return rc;
    for (int k = 0; k < MCMP2_NKERNELS; ++k) {
        if (total_ms) total_ms[k] = ms[k];
        if (launches) launches[k] = n[k];
    }
    return MCMP2_OK;
}

extern "C" void mcmp2_destroy(mcmp2_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}
