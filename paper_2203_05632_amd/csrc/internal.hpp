// Internal declarations shared by the translation units of libmcmp2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mcmp2.h"

typedef double d4v __attribute__((ext_vector_type(4)));

// Walker pairs are padded to a multiple of kWalkerPad so that the point
// dimension (2 per pair) tiles by 16 and the row dimension (8 per pair:
// 2 electrons x 4 spinor components) by 64.
constexpr int kWalkerPad = 8;
// Block tile of the Green's-function kernel: 4 pairs = 32 rows.
constexpr int kTileWalkers = 4;

// Event-pair timing of selected kernels (mcmp2_profile_begin/end).
struct Profiler {
    uint32_t mask = 0;
    int capacity = 0, used = 0;
    hipEvent_t *ev = nullptr;  // [capacity][2]
    int *kid = nullptr;        // [capacity]
};

struct mcmp2_ctx {
    int device = 0;
    int n_cu = 256;  // compute units of the device (queried at init)
    hipStream_t stream = nullptr;
    int n_nuc = 0, nL = 0, nS = 0, nb = 0;
    int no = 0, nv = 0, nsp = 0;
    int m = 0, m_pad = 0;
    int E = 0;      // padded number of points, 2 * m_pad
    int R = 0;      // padded number of spinor rows, 8 * m_pad; row = 8 p + 4 e + c
    int T = 0;      // walker tiles, m_pad / kTileWalkers
    int n_tp = 0;   // tile pairs P <= Q
    int n_tau_max = 0;
    int precision = MCMP2_FP64;
    int want_grad = 0;
    int interaction = MCMP2_COULOMB;  // mcmp2_set_interaction
    double lambda = 0.0, Ng = 0.0;

    // device memory
    double *nuc = nullptr;    // [n_nuc][3]
    double *gpar = nullptr;   // [n_nuc][4] = c1 N(z1), z1, c2 N(z2), z2
    double *pgeo = nullptr;   // [nb][4] centre x, y, z, exponent
    double *pnl = nullptr;    // [nb][2] normalisation, Cartesian powers lx | ly << 8 | lz << 16 (int64 bits)
    double *coef = nullptr;   // [2][nb][nsp] complex
    double *eps = nullptr;    // [nsp]
    double *XT = nullptr;     // [nb][E] basis values, point fastest (padding points stay zero)
    double *hinv = nullptr;   // [m_pad] N_g / (g(r1p) g(r2p))
    double *rhat = nullptr;   // [m_pad][4] unit vector of r1p - r2p (x, y, z, 0)
    double *psi = nullptr;    // [nsp][R] complex, row fastest (double2; float2 for low-precision modes)
    void *U = nullptr;        // low-precision modes: [n_tau_max][R][Ktot] scaled operands (see green_lp.hip)
    int Ko = 0, Ktot = 0;     // K extents of the occupied segment and of all spinors (reals, multiples of the K chunk)
    double *scale = nullptr;  // [n_tau_max][nsp] exp(+eps tau) occupied, exp(-eps tau) virtual
    double *wtau = nullptr;   // [n_tau_max]
    int *tiles = nullptr;     // [n_tp][2] (P, Q), P <= Q
    int *work = nullptr;      // [n_slots / 4] tile-pair index per block (-1: idle), XCD-aware order
    int n_slots = 0;          // partial-sum slots: 4 per block (one per wave)
    int T16 = 0, n_tp16 = 0;  // BF16 / FP16: 16-walker tiles per side, tile pairs P <= Q
    int *tiles16 = nullptr;   // [n_tp16][2] (P, Q) in 4 x 8 patches
    double *partial = nullptr;  // [n_tau_max][max(n_slots, 8 n_tp16)][2] per wave slot (direct, exchange)
    // gradient work space (allocated when want_grad)
    // adjoint blocks [n_tau_max][R][R]: complex FP64 (FP64, FP32 modes) or
    // packed BF16 pairs, real part in the low half (BF16, FP16 modes)
    double *Hm = nullptr;       // adjoint of G-
    double *Hp = nullptr;       // adjoint of G+
    double *psibar = nullptr;   // [nsp][R] complex gradient of psi (FP64, FP32 modes)
    uint32_t *Vt = nullptr;     // BF16 / FP16 modes: [n_tau_max][nsp][R] psi s_t as packed BF16 pairs
    // BF16 / FP16 modes: BF16 operands of the spinor GEMM and the coefficient
    // gradient (primitive sets padded to nLp, nSp = nbp - nLp; points padded
    // to Ep; all multiples of 64, padding zero)
    int nLp = 0, nbp = 0, Ep = 0;
    void *Cb = nullptr;   // [4 nsp][3 nbp]: row 4 k + 2 s + ri = part ri of C[s][mu][k], split [hi|hi|lo] per set
    void *Xb = nullptr;   // [E][3 nbp] basis values per point, split [hi|lo|hi] per set
    void *XTb = nullptr;  // [nb][Ep] basis values per primitive (gradients)
    void *PBb = nullptr;  // [2 sets][4 nsp][Ep] psi gradient (gradients), written by the adjoint GEMM
    double *eps_part = nullptr; // [row tiles][nsp] eps-gradient partials (32-row tiles, or 128-row in BF16 / FP16 modes)
    // BF16 / FP16 modes below one coefficient-gradient tile per two CUs: staging
    // of both gradients for mcmp2_step_accumulate ([nsp] rounded up to even,
    // then complex [2][nb][nsp]), which there adds them with separate launches
    double *gstage = nullptr;

    Profiler prof;
};

// Neumaier step: (s, c) += x with the rounding error of s + x kept in c.
__device__ inline void neumaier(double &s, double &c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Where a gradient goes: written to out, or (when sum is set) added to the
// compensated pair (sum, comp) element by element with neumaier().
struct grad_out {
    double *out = nullptr, *sum = nullptr, *comp = nullptr;
    bool any() const { return out || sum; }
};

// Work items of the spinor GEMMs: (primitive set, spinor tile, point tile).
// Block b runs on XCD b % 8; each XCD takes a contiguous range of the n_pairs
// (spinor tile, point tile) pairs and first runs their small-component
// items (the longer K loop), then the large-component ones, which fill in
// behind them (longest first; 16 ceil(n_pairs / 8) blocks).  Returns false
// for a padding block.
__device__ inline bool spinor_set_item(int n_pairs, int &set, int &pair) {
    const int pp = (n_pairs + 7) / 8, x = (int)(blockIdx.x % 8), j = (int)(blockIdx.x / 8);
    const int cnt = min(pp, n_pairs - x * pp);
    if (j >= 2 * cnt) return false;
    set = j < cnt ? 1 : 0;
    pair = x * pp + (j < cnt ? j : j - cnt);
    return true;
}

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

// g(r) of Eq. basisSet; gpar[I] = (c1 N(z1), z1, c2 N(z2), z2).
__device__ inline double g_value(double x, double y, double z, const double *nuc, const double *gpar, int n_nuc) {
    double out = 0.0;
    for (int I = 0; I < n_nuc; ++I) {
        double dx = x - nuc[3 * I], dy = y - nuc[3 * I + 1], dz = z - nuc[3 * I + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        out = out + gpar[4 * I] * exp(-gpar[4 * I + 1] * r2);
        out = out + gpar[4 * I + 2] * exp(-gpar[4 * I + 3] * r2);
    }
    return out;
}

// Item i of the per-step scalars, i in [0, m + n_tau nsp + n_tau): for a walker
// pair (i < m) the factor N_g / (g(r1) g(r2)) and the unit vector of r1 - r2;
// then the tau scalings exp(+eps_k tau_t) (occupied k) / exp(-eps_k tau_t)
// (virtual k); then the tau weights w(tau_t) = lambda exp(-lambda tau_t).
__device__ inline void prep_scalar_item(int i, const double *walkers, int m, const double *nuc, const double *gpar,
                                        int n_nuc, double Ng, double *hinv, double *rhat, const double *tau,
                                        const double *eps, int n_tau, int nsp, int no, double lambda, double *scale,
                                        double *wtau) {
    if (i < m) {
        const double *r = walkers + 6 * i;
        const double g1 = g_value(r[0], r[1], r[2], nuc, gpar, n_nuc);
        const double g2 = g_value(r[3], r[4], r[5], nuc, gpar, n_nuc);
        hinv[i] = Ng / (g1 * g2);
        const double dx = r[0] - r[3], dy = r[1] - r[4], dz = r[2] - r[5];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;  // coincident electrons: no direction
        rhat[4 * i] = dx * inv;
        rhat[4 * i + 1] = dy * inv;
        rhat[4 * i + 2] = dz * inv;
        rhat[4 * i + 3] = 0.0;
    } else if (i < m + n_tau * nsp) {
        const int j = i - m, t = j / nsp, k = j - t * nsp;
        const double tv = tau[t];
        scale[j] = k < no ? exp(eps[k] * tv) : exp(-eps[k] * tv);
    } else {
        const int t = i - m - n_tau * nsp;
        wtau[t] = lambda * exp(-lambda * tau[t]);
    }
}

// Event pair around a single kernel dispatch when kernel id `kid` is being
// timed (mcmp2_profile_begin): prof_begin() records the start event and
// returns the slot (-1 when not recording), prof_end() the stop event.  The
// launchers bracket their main GEMM dispatch with it (MCMP2_K_GREEN_GEMM,
// MCMP2_K_ADJ_GEMM), inside the stage-level pairs of the C ABI.
inline int prof_begin(const mcmp2_ctx *c, int kid) {
    Profiler &p = const_cast<Profiler &>(c->prof);
    if (!((p.mask >> kid) & 1u) || p.used >= p.capacity) return -1;
    const int slot = p.used;
    if (hipEventRecord(p.ev[2 * slot], c->stream) != hipSuccess) return -1;
    p.kid[slot] = -1;  // filled in by prof_end
    ++p.used;
    return slot;
}
inline hipError_t prof_end(const mcmp2_ctx *c, int slot, int kid) {
    if (slot < 0) return hipSuccess;
    Profiler &p = const_cast<Profiler &>(c->prof);
    hipError_t e = hipEventRecord(p.ev[2 * slot + 1], c->stream);
    if (e == hipSuccess) p.kid[slot] = kid;
    return e;
}

// Host: wave-slot work list of the Green's-function kernel (see green.hip).
void build_green_work(int T, double tile_bytes, std::vector<int> &work);

// Host set-up shared by mcmp2_init and mcmp2_step_noalloc (api.hip).
// check_setup validates the set-up arguments (EINVAL with a message) and
// returns lambda = 2 (eps_LUMO - eps_HOMO); setup_ctx fills the sizes,
// padding and frozen constants of a context (no device memory) and the
// weight-function records gpar; pack_basis packs the primitive records
// (A, zeta) and (N, Cartesian powers as int64 bits); triangle_tiles lists the
// walker-tile pairs P <= Q; green_tile_bytes is the operand bytes of one
// Green's-kernel block tile (the work-list builder's L2 model).
int check_setup(const mcmp2_basis *basis, const double *coeffs, const double *eps, int n_occ, int n_vir,
                int m_pairs, int n_tau_max, int precision, double *lambda_out);
int setup_ctx(mcmp2_ctx *c, const mcmp2_basis *basis, int n_occ, int n_vir, int m_pairs, int n_tau_max,
              int precision, int want_grad, double lambda, void *hip_stream, std::vector<double> &gpar);
void pack_basis(const mcmp2_basis *basis, std::vector<double> &geo, std::vector<double> &nl);
void triangle_tiles(int T, std::vector<int> &tiles);
double green_tile_bytes(const mcmp2_ctx *c);

// error reporting (thread-local message)
void set_error(const char *fmt, ...);
int check_hip(hipError_t e, const char *what);

// launchers (return hipError_t of the launch)
hipError_t launch_walker_weights(const mcmp2_ctx *c, const double *walkers, double *w, double *hinv);
hipError_t launch_metropolis(const mcmp2_ctx *c, double *walkers, double *w, uint64_t key0,
                             uint64_t key1, uint64_t step, double delta, int32_t *n_acc);
hipError_t launch_sample_tau(const mcmp2_ctx *c, uint64_t key0, uint64_t key1, uint64_t step,
                             int n_tau, double *tau);
hipError_t launch_advance(const mcmp2_ctx *c, double *walkers, double *w, uint64_t key0, uint64_t key1, uint64_t step,
                          double delta, int32_t *n_acc, int n_tau, double *tau);
hipError_t launch_step_prep(const mcmp2_ctx *c, const double *walkers, const double *tau, int n_tau);
hipError_t launch_spinor_gemm(const mcmp2_ctx *c);
hipError_t launch_green_contract(const mcmp2_ctx *c, int n_tau, bool grad);
// Tau samples per block (1 or 2, dividing n_tau) of the 32x32-tile FP64 and
// FP32 Green's kernels for a launch of nblocks tile pairs (makespan model).
int green_tau_chunk(int nblocks, int n_tau, int n_cu);
hipError_t launch_green_lp(const mcmp2_ctx *c, int n_tau, bool grad);
// BF16 / FP16: 128 x 128 block tiles (16 walkers a side) when they fill the GPU
bool green_big_selected(const mcmp2_ctx *c, int n_tau);
void build_big_tiles(int T16, std::vector<int> &tiles);
hipError_t launch_accumulate(const mcmp2_ctx *c, const double *src, double *sum, double *comp, int64_t n);
hipError_t launch_adjoint(const mcmp2_ctx *c, const double *tau, int n_tau, grad_out grad_eps);
hipError_t launch_coef_grad(const mcmp2_ctx *c, grad_out grad_coeffs);
hipError_t launch_adjoint_lp(const mcmp2_ctx *c, const double *tau, int n_tau);
// Gaunt / Breit adjoint blocks in the BF16 / FP16 modes (green.hip)
hipError_t launch_breit_adjoint_lp(const mcmp2_ctx *c, int n_tau, double cgrad);
hipError_t launch_coef_lp(const mcmp2_ctx *c);
hipError_t launch_spinor_lp(const mcmp2_ctx *c);
// true when the split-BF16 spinor GEMM has at least one 128x128 tile per two CUs
bool spinor_lp_tiled(const mcmp2_ctx *c);
// XT -> XTb (gradients) and, with want_xb, the split-BF16 operand Xb
hipError_t launch_x_lp(const mcmp2_ctx *c, bool want_xb);
// step_prep for the tiled BF16 / FP16 spinor GEMM: the basis values go straight
// to Xb (and XTb) without the FP64 XT, plus the per-step scalars
hipError_t launch_step_prep_lp(const mcmp2_ctx *c, const double *walkers, const double *tau, int n_tau);
hipError_t launch_coef_grad_lp(const mcmp2_ctx *c, grad_out grad_coeffs);
// whether the BF16 coefficient gradient adds into running sums itself (enough tiles to hide its loads)
bool coef_grad_lp_fused(const mcmp2_ctx *c);
int adjoint_lp_row_tiles(const mcmp2_ctx *c);
hipError_t launch_reduce(const mcmp2_ctx *c, int n_tau, double *e2_out);
// value[0] = (1/n_tau) sum_t e2_out[t][2]
hipError_t launch_step_value(const mcmp2_ctx *c, const double *e2_out, int n_tau, double *value);
