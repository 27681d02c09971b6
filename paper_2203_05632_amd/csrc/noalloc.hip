// mcmp2_step_noalloc: the FP64 estimator of mcmp2_step without a context and
// without any device allocation.  Every per-step buffer of the step (packed
// basis records, basis values, spinor values, tau scalings, work lists,
// per-wave partial sums) lives in one file-scope device array of fixed size;
// the caller's coefficients are read in place.
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace {

// Per-device scratch of the no-allocation entry point (32 MiB).
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up once per device.
// In host code the array's name is only a host-side stand-in, so kernels and
// copies use these addresses.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d outside 0..%d", device, kMaxDevices - 1);
        return MCMP2_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc != MCMP2_OK) return rc;
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return MCMP2_OK;
}

// Sub-buffers carved out of the scratch array, each 256-byte aligned.  With
// base == nullptr only the total size is computed.
struct Carver {
    unsigned char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// Lay the FP64 step's buffers out from `base`; returns the bytes used.  The
// regions that must read as zero where the kernels do not write them
// (padding points and rows) come first, so one fill clears [0, zero_bytes).
size_t carve(mcmp2_ctx *c, unsigned char *base, int n_tau, size_t n_work, size_t *zero_bytes) {
    Carver cv{base};
    c->XT = cv.take<double>((size_t)c->nb * c->E);
    c->psi = cv.take<double>(2 * (size_t)c->nsp * c->R);
    c->hinv = cv.take<double>((size_t)c->m_pad);
    c->rhat = cv.take<double>(4 * (size_t)c->m_pad);
    *zero_bytes = cv.off;
    c->nuc = cv.take<double>(3 * (size_t)c->n_nuc);
    c->gpar = cv.take<double>(4 * (size_t)c->n_nuc);
    c->pgeo = cv.take<double>(4 * (size_t)c->nb);
    c->pnl = cv.take<double>(2 * (size_t)c->nb);
    c->eps = cv.take<double>((size_t)c->nsp);
    c->scale = cv.take<double>((size_t)n_tau * c->nsp);
    c->wtau = cv.take<double>((size_t)n_tau);
    c->tiles = cv.take<int>(2 * (size_t)c->n_tp);
    c->work = cv.take<int>(n_work);
    c->partial = cv.take<double>((size_t)n_tau * c->n_slots * 2);
    return cv.off;
}

__global__ void zero_fill_kernel(double2 *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

}  // namespace

extern "C" int mcmp2_step_noalloc(const mcmp2_basis *basis, const double *coeffs, const double *eps, int32_t n_occ,
                                  int32_t n_vir, int32_t m_pairs, const double *walkers, const double *tau,
                                  int32_t n_tau, double *e2_out, double *value, void *hip_stream) {
    double lambda = 0.0;
    int rc = check_setup(basis, coeffs, eps, n_occ, n_vir, m_pairs, n_tau, MCMP2_FP64, &lambda);
    if (rc != MCMP2_OK) return rc;
    if (!walkers || !tau || !e2_out) {
        set_error("null argument");
        return MCMP2_EINVAL;
    }
    mcmp2_ctx c;  // host description only: every device pointer goes into the scratch array
    std::vector<double> gpar;
    if ((rc = setup_ctx(&c, basis, n_occ, n_vir, m_pairs, n_tau, MCMP2_FP64, 0, lambda, hip_stream, gpar)) !=
        MCMP2_OK)
        return rc;
    c.coef = const_cast<double *>(coeffs);  // read only by the spinor GEMM
    std::vector<int> tiles, work;
    triangle_tiles(c.T, tiles);
    build_green_work(c.T, green_tile_bytes(&c), work);
    c.n_slots = 4 * (int)work.size();
    size_t zero_bytes = 0;
    const size_t need = carve(&c, nullptr, n_tau, work.size(), &zero_bytes);
    if (need > kScratchBytes) {
        set_error("problem needs %zu bytes of scratch; mcmp2_step_noalloc holds at most %zu (m=%d, n_L+n_S=%d, "
                  "n_sp=%d, n_tau=%d)",
                  need, kScratchBytes, m_pairs, c.nb, c.nsp, n_tau);
        return MCMP2_EINVAL;
    }
    unsigned char *base = nullptr;
    if ((rc = scratch_address(c.device, &base)) != MCMP2_OK) return rc;
    carve(&c, base, n_tau, work.size(), &zero_bytes);

    std::vector<double> geo, nl;
    pack_basis(basis, geo, nl);
    // the array keeps the previous call's contents: clear the padding regions
    const size_t n2 = zero_bytes / sizeof(double2);
    zero_fill_kernel<<<(unsigned)std::min<size_t>((n2 + 255) / 256, 2048), 256, 0, c.stream>>>(
        reinterpret_cast<double2 *>(base), n2);
    if ((rc = check_hip(hipGetLastError(), "zero_fill")) != MCMP2_OK) return rc;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream), "hipMemcpyAsync");
    };
    if ((rc = up(c.nuc, basis->nuc_xyz, 3 * sizeof(double) * c.n_nuc)) != MCMP2_OK ||
        (rc = up(c.gpar, gpar.data(), gpar.size() * sizeof(double))) != MCMP2_OK ||
        (rc = up(c.pgeo, geo.data(), geo.size() * sizeof(double))) != MCMP2_OK ||
        (rc = up(c.pnl, nl.data(), nl.size() * sizeof(double))) != MCMP2_OK ||
        (rc = up(c.eps, eps, sizeof(double) * c.nsp)) != MCMP2_OK ||
        (rc = up(c.tiles, tiles.data(), tiles.size() * sizeof(int))) != MCMP2_OK ||
        (rc = up(c.work, work.data(), work.size() * sizeof(int))) != MCMP2_OK)
        return rc;
    if ((rc = check_hip(launch_step_prep(&c, walkers, tau, n_tau), "step_prep")) != MCMP2_OK ||
        (rc = check_hip(launch_spinor_gemm(&c), "spinor_gemm")) != MCMP2_OK ||
        (rc = check_hip(launch_green_contract(&c, n_tau, false), "green_contract")) != MCMP2_OK ||
        (rc = check_hip(launch_reduce(&c, n_tau, e2_out), "reduce")) != MCMP2_OK)
        return rc;
    if (value && (rc = check_hip(launch_step_value(&c, e2_out, n_tau, value), "step_value")) != MCMP2_OK) return rc;
    // the host staging above must outlive its copies
    return check_hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
}
