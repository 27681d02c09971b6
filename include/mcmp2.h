/*
 * mcmp2.h -- C ABI of the MI355X implementation of the per-step hot path of
 * stochastic four-component relativistic MP2 (Cruz, Garza, Yanai, Hirata,
 * arXiv 2203.05632, Sec. III).
 *
 * One MC step evaluates the redundant-walker estimator (Eq. redundant)
 *   I'_n = (1/mC2) sum_{p<q} f(r1p, r2p, r1q, r2q, tau) / (w(r1p,r2p) w(r1q,r2q) w(tau))
 * of the 13-dimensional integral that the Laplace transform turns Eq. FinalMP2
 * into.  Spinor values come from the basis expansion of Eq. (C); the integrand
 * is built from the 4x4 Green's functions G+ / G- (Sec. III) as
 *   f = -(1/2) (D - X) / (r12 r34),
 *   D = Tr[G-(3,1) G+(1,3)] Tr[G-(4,2) G+(2,4)],
 *   X = Tr[G-(3,1) G+(1,4) G-(4,2) G+(2,3)],
 * with G-(x,y) = sum_i phi_i(x) phi_i(y)^dagger exp(+eps_i tau) and
 * G+(x,y) = sum_a phi_a(x) phi_a(y)^dagger exp(-eps_a tau).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status codes: MCMP2_OK or a negative MCMP2_E*; mcmp2_last_error() then
 *   returns a thread-local message.  Nothing throws across the ABI.
 * - Host pointers are read during the call only (init copies them).
 *   Device pointers are caller-owned device memory; the library uses them on
 *   the context's HIP stream and never frees them.  Calls enqueue work and
 *   return without synchronising the host, except mcmp2_init and
 *   mcmp2_destroy.
 * - Complex arrays are interleaved (re, im) doubles.
 * - Spinor components are ordered (L alpha, L beta, S alpha, S beta).
 *   The paper prints one coefficient set C^L for both spins; this library
 *   takes one coefficient block per spin: coeffs[s][mu][k], s = 0 alpha,
 *   1 beta, mu over the L primitives then the S primitives.
 * - After MCMP2_EDEVICE the context must only be destroyed.
 */
#ifndef MCMP2_H
#define MCMP2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcmp2_ctx mcmp2_ctx; /* opaque; owns all of its device memory */

enum {
    MCMP2_OK = 0,
    MCMP2_EINVAL = -1, /* bad argument: shape, range or null pointer */
    MCMP2_ENOMEM = -2, /* device allocation failed */
    MCMP2_EDEVICE = -3, /* a HIP call failed */
    MCMP2_ESTATE = -4  /* call not valid in the context's state (e.g. gradients not enabled) */
};

/* Operand precision of the spinor and Green's-function contractions.
 * Exponential scalings, weights and all accumulations stay in FP64. */
enum { MCMP2_FP64 = 0, MCMP2_FP32 = 1, MCMP2_BF16 = 2, MCMP2_FP16 = 3 };
/* electron-electron interaction of the integrand (mcmp2_set_interaction) */
enum { MCMP2_COULOMB = 0, MCMP2_GAUNT = 1, MCMP2_BREIT = 2 };

/* Molecule, weight function and basis (host memory, caller-owned, copied by init). */
typedef struct {
    int32_t n_nuc;
    const double *nuc_xyz;    /* [n_nuc][3] nuclear positions, bohr */
    const double *wfn;        /* [n_nuc][4] = c1, zeta1, c2, zeta2 of Eq. basisSet (Table 1 form) */
    int32_t n_L, n_S;         /* Cartesian primitives of the large and small component sets */
    const double *prim_xyz;   /* [n_L+n_S][3] centres, L set first */
    const double *prim_exp;   /* [n_L+n_S] exponents (> 0) */
    const int32_t *prim_lxyz; /* [n_L+n_S][3] Cartesian powers, each in 0..4 */
    const double *prim_norm;  /* [n_L+n_S] normalisation constants */
} mcmp2_basis;

/*
 * mcmp2_init -- build a context for one walker set (Sec. III).
 *   basis      : see mcmp2_basis.
 *   coeffs     : host, complex [2][n_L+n_S][n_occ+n_vir], Eq. (C) coefficients.
 *   eps        : host, [n_occ+n_vir] spinor energies, occupied first.
 *   m_pairs    : number of electron-pair walkers m (>= 2), Eq. redundant.
 *   n_tau_max  : largest n_tau a step will be given (>= 1).
 *   precision  : MFMA operand types of the step's GEMMs, all with FP32
 *                accumulation outside FP64 mode:
 *                  mode   spinor GEMM     Green's GEMMs  contraction  adjoint GEMM  coefficient gradient
 *                  FP64   FP64            FP64           FP64         FP64          FP64
 *                  FP32   FP32            FP32           FP64         FP64          FP64
 *                  BF16   split BF16 (*)  BF16           FP32         BF16          BF16
 *                  FP16   split BF16 (*)  FP16           FP32         BF16          BF16
 *                (*) basis values and coefficients split as hi + lo BF16
 *                parts, three products (about 16 significant bits), when the
 *                GEMM has at least one 128x128 tile per two compute units;
 *                below that, FP32 (operands rounded from FP64).  The adjoint GEMM
 *                and coefficient gradient of FP16 mode use BF16 for its
 *                exponent range.  The contraction column is the type of the
 *                traces and 4x4 block products of the pair contraction.
 *                exp(+-eps tau) scalings (applied as square roots to both
 *                Green's-function operands, rounded once), pair weights and
 *                every sum stay in FP64.
 *   want_grad  : non-zero to allow gradient outputs in mcmp2_step and
 *                mcmp2_step_accumulate; allocates 2 n_tau_max (8 m_pad)^2
 *                complex adjoint matrices (FP64, or packed BF16 pairs in the
 *                BF16 / FP16 modes; m_pad = m rounded up to a multiple of 8)
 *                and, in the BF16 / FP16 modes of small problems, a staging
 *                copy of both gradients.
 *   hip_stream : hipStream_t to enqueue on (NULL = default stream).
 *   out        : receives the context.
 * lambda = 2 (eps_LUMO - eps_HOMO) (Eq. tauWeight and the rule after it) and
 * N_g (Sec. III, evaluated analytically from two-centre s-Gaussian Coulomb
 * integrals) are computed here and frozen.  All per-step buffers are
 * allocated here; mcmp2_step allocates nothing.
 * Errors: EINVAL (sizes, pointers, lambda <= 0), ENOMEM, EDEVICE.
 */
int mcmp2_init(const mcmp2_basis *basis, const double *coeffs, const double *eps, int32_t n_occ,
               int32_t n_vir, int32_t m_pairs, int32_t n_tau_max, int32_t precision, int32_t want_grad,
               void *hip_stream, mcmp2_ctx **out);

/*
 * mcmp2_step -- one evaluation of Eq. redundant at fixed walkers and tau.
 *   walkers : device [m][2][3] positions (r1p, r2p), bohr.
 *   tau     : device [n_tau] imaginary times (>= 0), 1 <= n_tau <= n_tau_max.
 *   e2_out  : device [n_tau][3]: per tau, the direct part Re(-D/2 ...), the
 *             exchange part Re(+X/2 ...) and their sum, each divided by
 *             w_p w_q w(tau) and averaged over the mC2 pairs p < q.
 *   value   : device [1] or NULL: the step value
 *             V = (1/n_tau) sum_t e2_out[t][2] (tau samples averaged at the
 *             same walkers), summed in tau order with compensation.
 *   grad_eps    : device [n_sp] or NULL.  dV/d eps_k of the step value
 *                 V = (1/n_tau) sum_t e2_out[t][2], at fixed walkers, tau and
 *                 lambda (lambda is a sampling parameter frozen at init).
 *   grad_coeffs : device complex [2][n_L+n_S][n_sp] or NULL; dV/dRe C + i dV/dIm C.
 *   Gradients overwrite their outputs.  Either requires want_grad at init
 *   (ESTATE otherwise); they come from a hand-written adjoint of the same
 *   step (Green's-function blocks recomputed, not stored between calls).
 * Errors: EINVAL (null pointers, n_tau out of range), ESTATE, EDEVICE.
 */
int mcmp2_step(mcmp2_ctx *ctx, const double *walkers, const double *tau, int32_t n_tau, double *e2_out,
               double *value, double *grad_eps, double *grad_coeffs);

/*
 * mcmp2_step_accumulate -- mcmp2_step with both gradients, each added to a
 * running compensated sum instead of written out: the same step value and
 * e2_out, and (eps_sum, eps_comp) and (coeffs_sum, coeffs_comp) end up
 * bit for bit as after mcmp2_step followed by mcmp2_accumulate of grad_eps
 * and of grad_coeffs (as 4 (n_L+n_S) n_sp doubles) into them, without the
 * gradient arrays being written and read back (the accumulation of the
 * gradient averages over MC steps, Eq. redundant).
 *   walkers, tau, n_tau, e2_out : as for mcmp2_step.
 *   eps_sum, eps_comp       : device [n_sp] doubles (compensated pair).
 *   coeffs_sum, coeffs_comp : device complex [2][n_L+n_S][n_sp] (as
 *                             grad_coeffs), 16-byte aligned.
 * The caller zeroes the pairs to start; the running total of a gradient is
 * sum + comp.
 * Errors: EINVAL (null pointers, n_tau out of range), ESTATE (context without
 * want_grad), EDEVICE.
 */
int mcmp2_step_accumulate(mcmp2_ctx *ctx, const double *walkers, const double *tau, int32_t n_tau, double *e2_out,
                          double *eps_sum, double *eps_comp, double *coeffs_sum, double *coeffs_comp);

/*
 * mcmp2_set_coefficients -- replace the context's spinor coefficients and
 * energies (Eq. (C), Eq. FinalMP2) with device arrays of the init layout:
 *   coeffs : device complex [2][n_L+n_S][n_sp];  eps : device [n_sp].
 * Copied on the context's stream (stream-ordered, no host sync).  lambda and
 * N_g stay as frozen at init.  Either pointer may be NULL to keep that array.
 * Errors: EINVAL (null context), EDEVICE.
 */
int mcmp2_set_coefficients(mcmp2_ctx *ctx, const double *coeffs, const double *eps);

/*
 * mcmp2_set_interaction -- choose the electron-electron interaction of the
 * integrand for the following steps.  Sec. II of the paper gives the operator
 *   g(1,2) = 1/r12 - alpha(1).alpha(2) / (2 r12)
 *            - (alpha(1).r12)(alpha(2).r12) / (2 r12^3)
 * (alpha: the Dirac matrices of Eq. alpha acting on each electron's four
 * components) and keeps only its first, Coulomb term, which is the default:
 *   MCMP2_COULOMB  1/r12 (the paper's runs)
 *   MCMP2_GAUNT    1/r12 - alpha(1).alpha(2) / (2 r12)
 *   MCMP2_BREIT    the full operator above.
 * With alpha inserted, the direct and exchange traces of the integrand carry
 * a Dirac matrix next to every Green's-function factor at the point it acts
 * on, weighted per walker pair by the 4x4 coefficients of g in the basis
 * (1, alpha_x, alpha_y, alpha_z) x (1, alpha_x, alpha_y, alpha_z).
 * The step's outputs keep their meaning (direct, exchange, total of the
 * estimator).  The Gaunt and Breit terms are evaluated in every precision
 * mode, the alpha-weighted contraction in FP64 on the mode's Green's
 * functions (in the BF16 / FP16 modes through the 32 x 32-tile Green's
 * kernel at every size).  Gradient outputs are available with them in every
 * mode: the adjoint of the alpha-weighted contraction is formed in FP64 from
 * the pairs' Green's-function blocks (kept as BF16 pairs in the BF16 / FP16
 * modes), and the adjoint GEMMs are those of the Coulomb interaction.
 * Errors: EINVAL (null context, unknown kind).
 */
int mcmp2_set_interaction(mcmp2_ctx *ctx, int32_t interaction);

/*
 * mcmp2_pair_weights -- w(r1p, r2p) = g(r1p) g(r2p) / (N_g r12p) for every
 * walker (Sec. III); the Metropolis chain needs it once at its start.
 *   walkers : device [m][2][3];  w : device [m] output.
 */
int mcmp2_pair_weights(mcmp2_ctx *ctx, const double *walkers, double *w);

/*
 * mcmp2_metropolis -- one Metropolis proposal per walker pair (Sec. III).
 * Both electrons of pair p move jointly, each coordinate by
 * delta * (2u - 1); the move is accepted iff u_acc < w(new)/w(old).
 * Uniforms come from Philox4x64-10 (Salmon et al., SC'11) with key
 * (key0, key1) and counter (step, p, purpose, 0): words 0-3 of purpose 0 and
 * words 0-1 of purpose 1 are the six displacement uniforms (r1 x,y,z then
 * r2 x,y,z), word 2 of purpose 1 is u_acc; a word u maps to (u >> 11) 2^-53.
 *   walkers    : device [m][2][3], updated in place.
 *   w          : device [m] current pair weights, updated in place.
 *   n_accepted : device int32, incremented by the number of accepted moves
 *                (may be NULL).
 * Errors: EINVAL (null pointers, delta not finite or <= 0), EDEVICE.
 */
int mcmp2_metropolis(mcmp2_ctx *ctx, double *walkers, double *w, uint64_t key0, uint64_t key1,
                     uint64_t step, double delta, int32_t *n_accepted);

/*
 * mcmp2_sample_tau -- n_tau imaginary times by the inverse CDF of
 * w(tau) = lambda exp(-lambda tau) (Sec. III): tau_t = -ln(1 - u_t) / lambda
 * with u_t word 0 of Philox counter (step, t, 2, 0), key (key0, key1).
 *   tau : device [n_tau] output.
 */
int mcmp2_sample_tau(mcmp2_ctx *ctx, uint64_t key0, uint64_t key1, uint64_t step, int32_t n_tau,
                     double *tau);

/*
 * mcmp2_advance -- mcmp2_metropolis followed by mcmp2_sample_tau for the same
 * (key, step), in one kernel launch: identical results to the two calls.
 *   walkers, w, n_accepted : as in mcmp2_metropolis;  tau : device [n_tau] output.
 * Errors: EINVAL (null pointers, delta not finite or <= 0, n_tau < 1), EDEVICE.
 */
int mcmp2_advance(mcmp2_ctx *ctx, double *walkers, double *w, uint64_t key0, uint64_t key1, uint64_t step,
                  double delta, int32_t *n_accepted, int32_t n_tau, double *tau);

/*
 * mcmp2_accumulate -- compensated (Neumaier) accumulation across MC steps:
 * for i < n, (sum[i], comp[i]) += src[i], so that sum[i] + comp[i] carries the
 * running total of every src added since the pair was zeroed (per-step E2
 * parts, eps gradients or, as 2 n doubles, complex coefficient gradients).
 *   src, sum, comp : device [n] doubles; n >= 0.  The caller zeroes sum and
 *   comp to start; calls are ordered on the context's stream.
 * Errors: EINVAL (null pointers with n > 0, n < 0), EDEVICE.
 */
int mcmp2_accumulate(mcmp2_ctx *ctx, const double *src, double *sum, double *comp, int64_t n);

/*
 * mcmp2_constants -- host copies of the frozen sampling constants.
 *   lambda, n_g : host outputs (either may be NULL).
 */
int mcmp2_constants(const mcmp2_ctx *ctx, double *lambda, double *n_g);

/*
 * Kernel timing with HIP events recorded on the context's stream, for
 * measurement harnesses.  mcmp2_profile_begin(ctx, mask, max_launches)
 * starts recording a start/stop event pair around every launch of the
 * kernels selected by `mask` (bit i = kernel id i below), for at most
 * max_launches launches in total (later launches run untimed).  Ids 0-10
 * time a stage of a call (which may enqueue several kernels); ids 11-12
 * time each dispatch of one kernel, so their launch counts are dispatches.
 * mcmp2_profile_end synchronises the stream, writes per-kernel total
 * milliseconds and launch counts into host arrays of length MCMP2_NKERNELS
 * (either may be NULL) and stops recording.
 * Errors: EINVAL (max_launches < 1), ESTATE (end without begin), ENOMEM, EDEVICE.
 */
enum {
    MCMP2_K_WALKER_WEIGHTS = 0, /* mcmp2_pair_weights */
    MCMP2_K_STEP_PREP = 1,      /* basis values, walker factors, tau scalings */
    MCMP2_K_SPINOR_GEMM = 2,    /* Eq. (C) */
    MCMP2_K_GREEN_CONTRACT = 3, /* G-/G+ and the pair contraction */
    MCMP2_K_REDUCE = 4,         /* compensated pair sums */
    MCMP2_K_METROPOLIS = 5,     /* mcmp2_metropolis */
    MCMP2_K_SAMPLE_TAU = 6,     /* mcmp2_sample_tau */
    MCMP2_K_ADVANCE = 7,        /* mcmp2_advance */
    MCMP2_K_GRAD = 8,           /* adjoint GEMM: psi and eps gradients */
    MCMP2_K_ACCUMULATE = 9,     /* mcmp2_accumulate */
    MCMP2_K_COEF_GRAD = 10,     /* coefficient gradient from the psi gradient */
    /* single dispatches inside the stages above (one pair per dispatch) */
    MCMP2_K_GREEN_GEMM = 11,    /* the Green's-function GEMM + contraction kernel itself */
    MCMP2_K_ADJ_GEMM = 12,      /* the adjoint GEMM kernel itself */
    MCMP2_NKERNELS = 13
};
int mcmp2_profile_begin(mcmp2_ctx *ctx, uint32_t mask, int32_t max_launches);
int mcmp2_profile_end(mcmp2_ctx *ctx, double *total_ms, int64_t *launches);

/*
 * mcmp2_step_noalloc -- for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): mcmp2_step of an
 * FP64 context with the Coulomb interaction and no gradients, without a
 * context.  It makes no device allocation: the step's buffers (packed basis
 * records, basis values, spinor values, tau scalings, work lists, per-wave
 * partial sums) live in a fixed 32 MiB device array of the library, one per
 * device, held until the process ends.
 *   basis, eps, n_occ, n_vir, m_pairs : as for mcmp2_init (host memory, read
 *                 during the call).
 *   coeffs      : DEVICE complex [2][n_L+n_S][n_occ+n_vir] (the layout of
 *                 mcmp2_init's coeffs), read in place.
 *   walkers, tau, n_tau, e2_out, value : as for mcmp2_step (device); n_tau >= 1.
 *   hip_stream  : hipStream_t to enqueue on (NULL = default stream).
 * Results equal mcmp2_step's on an FP64 context built from the same inputs.
 * The call synchronises hip_stream before returning.  Every call on a device
 * shares that device's array, and the array keeps the last call's contents
 * (the call clears what must start at zero): calls that overlap on one
 * device, from several threads or streams, race.
 * Errors: EINVAL (as mcmp2_init and mcmp2_step; a problem whose buffers
 * exceed the 32 MiB array, e.g. m = 128 walker pairs with 660 primitives and
 * 340 spinors needs about 7 MB), EDEVICE.
 */
int mcmp2_step_noalloc(const mcmp2_basis *basis, const double *coeffs, const double *eps, int32_t n_occ,
                       int32_t n_vir, int32_t m_pairs, const double *walkers, const double *tau, int32_t n_tau,
                       double *e2_out, double *value, void *hip_stream);

/* Release the context and its device memory (synchronises its stream). NULL is ignored. */
void mcmp2_destroy(mcmp2_ctx *ctx);

/* Thread-local message describing the last non-OK status ("" if none). */
const char *mcmp2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCMP2_H */
