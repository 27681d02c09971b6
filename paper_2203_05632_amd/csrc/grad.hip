// Gradients of the per-step value with respect to the spinor energies and
// coefficients (reverse mode through Eq. (C) and the G+ / G- definitions of
// Sec. III of the paper).
//
// The step value is V = (1/n_tau) sum_t (1/mC2) sum_{p<q} Re f / (w_p w_q w_t).
// The Green's-function kernel, in its GRAD variant, leaves for every tau the
// Hermitian adjoint matrices H-_t, H+_t (R x R complex): the gradient of V with
// respect to each entry of G-_t / G+_t, folded as Gbar + Gbar^H.  Since
// G_t = Psi S_t Psi^H with S_t = diag(exp(+eps tau)) (occupied) or
// diag(exp(-eps tau)) (virtual),
//   Psibar = sum_t H_t Psi S_t                                  (grad_gemm)
//   epsbar_k = (1/2) sum_t (+-tau_t) Re(psi_k^H (H_t Psi S_t)_k) (grad_gemm + eps_reduce)
// (the 1/2: dV/ds_k = Re(psi_k^H Gbar psi_k) = psi_k^H H psi_k / 2 for H = Gbar + Gbar^H)
//   Cbar[s][mu][k] = sum_pt chi_mu(r_pt) Psibar[k][4 pt + c(s, mu)]   (coef_grad)
// with the PyTorch convention dV/dRe + i dV/dIm for complex gradients.
#include <algorithm>

#include <type_traits>

#include "internal.hpp"

namespace {

constexpr int GKC = 16;  // rows y of H (and of psi) per LDS chunk
constexpr int kPadRow = 33;  // LDS row length (double2) of the 32-wide chunks

// Work items: (row tile of 32 rows x, column tile of 32 spinors: occupied
// tiles first, then virtual), in groups of kRowGroup row tiles; within a
// group, column-major, so that consecutive items share H row panels and psi
// column panels.  Block b runs on XCD b % 8, and each XCD takes a contiguous
// range of items: the blocks resident on one XCD at a time cover a few row
// panels x a few column panels and share them through that XCD's L2.
constexpr int kRowGroup = 8;

__device__ inline bool grad_item(int n_rt, int n_ct, int &rt, int &ct) {
    const int n_items = n_rt * n_ct, per = (n_items + 7) / 8;
    const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= n_items) return false;
    const int g = item / (kRowGroup * n_ct);
    const int rows = min(kRowGroup, n_rt - g * kRowGroup);
    const int w = item - g * kRowGroup * n_ct;
    ct = w / rows;
    rt = g * kRowGroup + w % rows;
    return true;
}

// grid: 8 ceil(n_rt n_ct / 8) blocks over the work items above (n_rt = R / 32
// row tiles, n_ct column tiles).  4 waves: 16x16 output sub-tiles (wx, wk).
// Psibar[k][x] = sum_t s_t[k] sum_y H_t[x][y] psi[k][y]; the partial
// epsbar of this row tile goes to eps_part[row tile][k].  The complex
// products take three real MFMA products (3M / Gauss form): for
// H = a + ib and s psi = c + id,
//   T1 = sum a c,  T2 = sum b d,  T3 = sum (a + b)(c + d),
//   Re = T1 - T2,  Im = T3 - T1 - T2.
__device__ inline double2 to_d2(const double2 &v) { return v; }
__device__ inline double2 to_d2(const float2 &v) { return double2{(double)v.x, (double)v.y}; }

typedef float f2v __attribute__((ext_vector_type(2)));

// P: element type of psi (double2 in FP64 mode, float2 in the low-precision modes)
template <int NT, typename P>
__global__ __launch_bounds__(256) void grad_gemm_kernel(
    const double2 *__restrict__ Hm, const double2 *__restrict__ Hp, const P *__restrict__ psi,
    const double *__restrict__ scale, const double *__restrict__ tau, int t0, int R, int no, int nsp, int n_occ_tiles,
    int n_col_tiles, bool accumulate, double2 *__restrict__ psibar, double *__restrict__ eps_part) {
    // H_t chunk [y][x] and psi chunk [y][k], rows padded to 33 entries (528 B):
    // the staging stores run down a column (16 lanes, consecutive y), which
    // with 512-byte rows would all hit the same four banks
    __shared__ double2 pa[2][NT][GKC][kPadRow];
    __shared__ double2 pb[2][GKC][kPadRow];
    __shared__ double esum[2][32];
    int rt, ct;
    if (!grad_item(R / 32, n_col_tiles, rt, ct)) return;  // padding block (the whole block)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wx = wave >> 1, wk = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    const bool occ = ct < n_occ_tiles;
    const int k0 = occ ? 32 * ct : no + 32 * (ct - n_occ_tiles);
    const int k_hi = occ ? no : nsp;
    const double sign = occ ? 1.0 : -1.0;
    const double2 *H = occ ? Hm : Hp;
    const int x0 = 32 * rt;
    const size_t RR = (size_t)R * R;

    // this lane's column k and its scalings s_t[k]
    const int kl = k0 + 16 * wk + li;
    const bool k_ok = kl < k_hi;
    double s[NT];
    for (int t = 0; t < NT; ++t) s[t] = k_ok ? scale[(size_t)(t0 + t) * nsp + kl] : 0.0;

    // cooperative chunk loads: element e in {tid, tid + 256} -> (row = e / 16, y = e % 16)
    const int e0 = tid, e1 = tid + 256;
    // staging registers as ext_vector_type (HIP's double2 struct would be kept in scratch memory)
    typedef double d2v __attribute__((ext_vector_type(2)));
    // FP32 psi: rows past k_hi are loaded clamped (always in bounds) and zeroed
    // when staged, so the load is unconditional and its wait (with the FP32 ->
    // FP64 conversion) falls at the LDS store after the chunk's MFMAs; loaded
    // under a condition, the conversion's wait sat right behind the chunk's
    // loads and drained the prefetch.  FP64 psi keeps the conditional load
    // (measured slightly faster there).
    constexpr bool F32 = std::is_same<P, float2>::value;
    using PV = typename std::conditional<F32, f2v, d2v>::type;
    d2v ra[NT][2];
    PV rb[2];
    auto gload = [&](int y0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int e = j ? e1 : e0, r = e >> 4, y = y0 + (e & 15);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                ra[t][j] = *reinterpret_cast<const d2v *>(&H[(size_t)(t0 + t) * RR + (size_t)(x0 + r) * R + y]);
            if constexpr (F32) {
                rb[j] = *reinterpret_cast<const PV *>(&psi[(size_t)min(k0 + r, k_hi - 1) * R + y]);
            } else {
                const int kk = k0 + r;
                const double2 pv = kk < k_hi ? psi[(size_t)kk * R + y] : double2{0.0, 0.0};
                rb[j] = d2v{pv.x, pv.y};
            }
        }
    };
    auto lstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int e = j ? e1 : e0, r = e >> 4, y = e & 15;
#pragma unroll
            for (int t = 0; t < NT; ++t) *reinterpret_cast<d2v *>(&pa[buf][t][y][r]) = ra[t][j];
            if constexpr (F32)
                *reinterpret_cast<d2v *>(&pb[buf][y][r]) =
                    k0 + r < k_hi ? d2v{(double)rb[j].x, (double)rb[j].y} : d2v{0.0, 0.0};
            else
                *reinterpret_cast<d2v *>(&pb[buf][y][r]) = rb[j];
        }
    };

    d4v t1[NT], t2[NT], t3[NT];
    for (int t = 0; t < NT; ++t) t1[t] = t2[t] = t3[t] = d4v{0.0, 0.0, 0.0, 0.0};
    const int n_chunks = R / GKC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < n_chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < n_chunks) gload((c + 1) * GKC);
        for (int ks = 0; ks < GKC; ks += 4) {
            const double2 bv = pb[buf][ks + lk][16 * wk + li];
            const double bs = bv.x + bv.y;
            for (int t = 0; t < NT; ++t) {
                const double2 av = pa[buf][t][ks + lk][16 * wx + li];
                const double c_ = bv.x * s[t], d_ = bv.y * s[t], cd = bs * s[t];
                t1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, c_, t1[t], 0, 0, 0);
                t2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, d_, t2[t], 0, 0, 0);
                t3[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x + av.y, cd, t3[t], 0, 0, 0);
            }
        }
        if (c + 1 < n_chunks) lstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: lane holds rows x = x0 + 16 wx + 4 v + lk, column kl
    double e_acc = 0.0;
    for (int v = 0; v < 4; ++v) {
        const int x = x0 + 16 * wx + 4 * v + lk;
        double yr = 0.0, yi = 0.0, re[NT], im[NT];
        for (int t = 0; t < NT; ++t) {
            re[t] = t1[t][v] - t2[t][v];
            im[t] = (t3[t][v] - t1[t][v]) - t2[t][v];
            yr += re[t];
            yi += im[t];
        }
        if (k_ok) {
            const double2 ph = to_d2(psi[(size_t)kl * R + x]);
            for (int t = 0; t < NT; ++t)  // Re(conj(psi) Y_t) weighted by +-tau_t / 2
                e_acc += 0.5 * sign * tau[t0 + t] * (ph.x * re[t] + ph.y * im[t]);
            double2 *o = psibar + (size_t)kl * R + x;
            if (accumulate) {
                const double2 old = *o;
                yr += old.x;
                yi += old.y;
            }
            *o = double2{yr, yi};
        }
    }
    // column sums over the 16 rows of the wave (lanes l, l^16, l^32, l^48), then the two row halves
    e_acc += __shfl_xor(e_acc, 16, 64);
    e_acc += __shfl_xor(e_acc, 32, 64);
    if (lk == 0) esum[wx][16 * wk + li] = e_acc;
    __syncthreads();
    if (tid < 32 && k0 + tid < k_hi) {
        double *o = eps_part + (size_t)rt * nsp + k0 + tid;
        const double v = esum[0][tid] + esum[1][tid];
        *o = accumulate ? *o + v : v;
    }
}

// epsbar[k] = sum over row tiles of eps_part, in row-tile order; written to
// grad_eps or added to (sum, comp).
__global__ void eps_reduce_kernel(const double *__restrict__ eps_part, int n_rowtiles, int nsp,
                                  double *__restrict__ grad_eps, double *__restrict__ sum,
                                  double *__restrict__ comp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsp) return;
    double acc = 0.0;
#pragma unroll 8  // loads of 8 row tiles in flight together; the adds keep their order
    for (int r = 0; r < n_rowtiles; ++r) acc += eps_part[(size_t)r * nsp + k];
    if (sum) {
        double sv = sum[k], cv = comp[k];
        neumaier(sv, cv, acc);
        sum[k] = sv;
        comp[k] = cv;
    } else {
        grad_eps[k] = acc;
    }
}

// Cbar[s][mu][k] = sum_pt XT[mu][pt] psibar[k][4 pt + 2 set(mu) + s].
// grid: (mu tiles of 16: L set first, then S set; ceil(nsp / 16)); 4 waves
// split the point range, wave 0 adds the partial tiles in a fixed order.
__global__ __launch_bounds__(256) void coef_grad_kernel(const double *__restrict__ XT, const double2 *__restrict__ psibar,
                                                        int E, int n_pts, int nb, int nL, int nsp, int R,
                                                        int n_L_tiles, double2 *__restrict__ grad_coeffs,
                                                        double2 *__restrict__ sum, double2 *__restrict__ comp) {
    __shared__ d4v red[3][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const bool setL = (int)blockIdx.x < n_L_tiles;
    const int mu0 = setL ? 16 * blockIdx.x : nL + 16 * (blockIdx.x - n_L_tiles);
    const int mu_hi = setL ? nL : nb;
    const int cbase = setL ? 0 : 2;
    const int k0 = 16 * blockIdx.y;
    const int mu = mu0 + li;
    const int kB = k0 + li;  // column of this lane's B element
    const bool mu_ok = mu < mu_hi, kB_ok = kB < nsp;
    d4v acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int pt0 = 4 * wave; pt0 < n_pts; pt0 += 16) {
        const int pt = pt0 + lk;
        const bool ok = pt < n_pts;
        const double x = (ok && mu_ok) ? XT[(size_t)mu * E + pt] : 0.0;
        double2 ba = {0.0, 0.0}, bb = {0.0, 0.0};
        if (ok && kB_ok) {
            ba = psibar[(size_t)kB * R + 4 * pt + cbase];
            bb = psibar[(size_t)kB * R + 4 * pt + cbase + 1];
        }
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, ba.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, ba.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, bb.x, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, bb.y, acc[3], 0, 0, 0);
    }
    if (wave > 0)
        for (int q = 0; q < 4; ++q) red[wave - 1][q][lane] = acc[q];
    __syncthreads();
    if (wave != 0) return;
    for (int w = 0; w < 3; ++w)
        for (int q = 0; q < 4; ++q) acc[q] += red[w][q][lane];
    // result D[4 v + lk][li]: row mu = mu0 + 4 v + lk, column k = k0 + li
    const int k = k0 + li;
    if (k >= nsp) return;
    for (int v = 0; v < 4; ++v) {
        const int mr = mu0 + 4 * v + lk;
        if (mr >= mu_hi) continue;
        const size_t ia = (size_t)mr * nsp + k, ib = ((size_t)nb + mr) * nsp + k;  // alpha, beta
        if (sum) {
            double2 sa = sum[ia], ca = comp[ia], sb = sum[ib], cb = comp[ib];
            neumaier(sa.x, ca.x, acc[0][v]);
            neumaier(sa.y, ca.y, acc[1][v]);
            neumaier(sb.x, cb.x, acc[2][v]);
            neumaier(sb.y, cb.y, acc[3][v]);
            sum[ia] = sa;
            comp[ia] = ca;
            sum[ib] = sb;
            comp[ib] = cb;
        } else {
            grad_coeffs[ia] = double2{acc[0][v], acc[1][v]};
            grad_coeffs[ib] = double2{acc[2][v], acc[3][v]};
        }
    }
}

// Large problems: 64 mu x 64 k output tiles (4 waves of 32 x 32, each 2 x 2
// MFMA sub-tiles for the four components alpha re, alpha im, beta re, beta
// im), points in chunks of CGK through LDS (double-buffered, the next chunk
// prefetched into registers): As[pt][mu] from XT, Bs[pt][component][k] from
// psibar.  Rows are padded by two doubles so that the four 128-byte row
// segments of one MFMA operand read fall in different banks.  Work items
// (mu tile, k tile), mu-tile major, are dealt to the XCDs in contiguous ranges
// (block b runs on XCD b % 8): blocks sharing XT rows read them through one L2.
constexpr int CGK = 8;        // points per chunk
constexpr int CGT = 64;       // mu and k per block tile
constexpr int CGP = CGT + 2;  // padded LDS row (doubles)

__global__ __launch_bounds__(256) void coef_grad_tile_kernel(const double *__restrict__ XT,
                                                             const double2 *__restrict__ psibar, int E, int n_pts,
                                                             int nb, int nL, int nsp, int R, int n_L_tiles,
                                                             int n_k_tiles, int n_items,
                                                             double2 *__restrict__ grad_coeffs,
                                                             double2 *__restrict__ sum, double2 *__restrict__ comp) {
    __shared__ __align__(16) double As[2][CGK][CGP];
    __shared__ __align__(16) double Bs[2][CGK][4][CGP];
    const int per = (n_items + 7) / 8;
    const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= n_items) return;
    const int mt = item / n_k_tiles, kt = item % n_k_tiles;
    const bool setL = mt < n_L_tiles;
    const int mu0 = setL ? CGT * mt : nL + CGT * (mt - n_L_tiles);
    const int mu_hi = setL ? nL : nb;
    const int cbase = setL ? 0 : 2;  // psibar index 4 pt + 2 set + s
    const int k0 = CGT * kt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wk = wave & 1, li = lane & 15, lk = lane >> 4;

    // staging: A element e = tid + 256 j (j < 2): mu e / 8, point e % 8;
    //          B pair e = tid + 256 j (j < 4): k e / 16, point (e / 2) % 8, spin e % 2
    double ra[2];
    double2 rb[4];
    auto gload = [&](int p0) __attribute__((always_inline)) {
        for (int j = 0; j < 2; ++j) {
            const int e = tid + 256 * j, mu = mu0 + e / 8, pt = p0 + e % 8;
            ra[j] = (mu < mu_hi && pt < n_pts) ? XT[(size_t)mu * E + pt] : 0.0;
        }
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j, k = k0 + e / 16, pt = p0 + (e / 2) % 8, sp = e % 2;
            rb[j] = (k < nsp && pt < n_pts) ? psibar[(size_t)k * R + 4 * pt + cbase + sp] : double2{0.0, 0.0};
        }
    };
    auto lstore = [&](int buf) __attribute__((always_inline)) {
        for (int j = 0; j < 2; ++j) {
            const int e = tid + 256 * j;
            As[buf][e % 8][e / 8] = ra[j];
        }
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j, kl = e / 16, pl = (e / 2) % 8, sp = e % 2;
            Bs[buf][pl][2 * sp][kl] = rb[j].x;
            Bs[buf][pl][2 * sp + 1][kl] = rb[j].y;
        }
    };
    d4v acc[2][2][4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int c = 0; c < 4; ++c) acc[i][j][c] = d4v{0.0, 0.0, 0.0, 0.0};
    const int n_chunks = (n_pts + CGK - 1) / CGK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < n_chunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < n_chunks) gload(CGK * (ch + 1));
#pragma unroll
        for (int ks = 0; ks < CGK; ks += 4) {
            double a[2], b[2][4];
            for (int i = 0; i < 2; ++i) a[i] = As[buf][ks + lk][32 * wm + 16 * i + li];
            for (int j = 0; j < 2; ++j)
                for (int c = 0; c < 4; ++c) b[j][c] = Bs[buf][ks + lk][c][32 * wk + 16 * j + li];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int c = 0; c < 4; ++c)
                        acc[i][j][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j][c], acc[i][j][c], 0, 0, 0);
        }
        if (ch + 1 < n_chunks) lstore(buf ^ 1);
        __syncthreads();
    }
    // result element v of sub-tile (i, j): mu = mu0 + 32 wm + 16 i + 4 v + lk, k = k0 + 32 wk + 16 j + li
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = k0 + 32 * wk + 16 * j + li;
            if (k >= nsp) continue;
            if (sum) {
                // the four elements' running sums are all loaded before any is updated
                // (loaded one at a time, each load waited for the previous stores)
                double2 sa[4], ca[4], sb[4], cb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int mr = min(mu0 + 32 * wm + 16 * i + 4 * v + lk, mu_hi - 1);
                    const size_t ia = (size_t)mr * nsp + k, ib = ((size_t)nb + mr) * nsp + k;  // alpha, beta
                    sa[v] = sum[ia];
                    ca[v] = comp[ia];
                    sb[v] = sum[ib];
                    cb[v] = comp[ib];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int mr = mu0 + 32 * wm + 16 * i + 4 * v + lk;
                    if (mr >= mu_hi) continue;
                    const size_t ia = (size_t)mr * nsp + k, ib = ((size_t)nb + mr) * nsp + k;
                    neumaier(sa[v].x, ca[v].x, acc[i][j][0][v]);
                    neumaier(sa[v].y, ca[v].y, acc[i][j][1][v]);
                    neumaier(sb[v].x, cb[v].x, acc[i][j][2][v]);
                    neumaier(sb[v].y, cb[v].y, acc[i][j][3][v]);
                    sum[ia] = sa[v];
                    comp[ia] = ca[v];
                    sum[ib] = sb[v];
                    comp[ib] = cb[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int mr = mu0 + 32 * wm + 16 * i + 4 * v + lk;
                    if (mr >= mu_hi) continue;
                    const size_t ia = (size_t)mr * nsp + k, ib = ((size_t)nb + mr) * nsp + k;  // alpha, beta
                    grad_coeffs[ia] = double2{acc[i][j][0][v], acc[i][j][1][v]};
                    grad_coeffs[ib] = double2{acc[i][j][2][v], acc[i][j][3][v]};
                }
            }
        }
}

template <typename P>
hipError_t launch_grad_gemm(const mcmp2_ctx *c, const double *tau, int n_tau, int n_occ_tiles, int n_vir_tiles) {
    const double2 *Hm = reinterpret_cast<const double2 *>(c->Hm), *Hp = reinterpret_cast<const double2 *>(c->Hp);
    const P *psi = reinterpret_cast<const P *>(c->psi);
    double2 *psibar = reinterpret_cast<double2 *>(c->psibar);
    const int n_ct = n_occ_tiles + n_vir_tiles;
    const int grid = 8 * ((c->R / 32 * n_ct + 7) / 8);
    for (int t0 = 0; t0 < n_tau; t0 += 2) {
        const int nt = std::min(2, n_tau - t0);
        const bool acc = t0 > 0;
        const int ps = prof_begin(c, MCMP2_K_ADJ_GEMM);
        if (nt == 2)
            grad_gemm_kernel<2, P><<<grid, 256, 0, c->stream>>>(Hm, Hp, psi, c->scale, tau, t0, c->R, c->no, c->nsp,
                                                                n_occ_tiles, n_ct, acc, psibar, c->eps_part);
        else
            grad_gemm_kernel<1, P><<<grid, 256, 0, c->stream>>>(Hm, Hp, psi, c->scale, tau, t0, c->R, c->no, c->nsp,
                                                                n_occ_tiles, n_ct, acc, psibar, c->eps_part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if ((e = prof_end(c, ps, MCMP2_K_ADJ_GEMM)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_adjoint(const mcmp2_ctx *c, const double *tau, int n_tau, grad_out grad_eps) {
    const int n_occ_tiles = (c->no + 31) / 32, n_vir_tiles = (c->nsp - c->no + 31) / 32;
    const bool h16 = c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16;
    const int n_rowtiles = h16 ? adjoint_lp_row_tiles(c) : c->R / 32;
    {
        hipError_t e = c->precision == MCMP2_FP64 ? launch_grad_gemm<double2>(c, tau, n_tau, n_occ_tiles, n_vir_tiles)
                       : h16                     ? launch_adjoint_lp(c, tau, n_tau)
                                                 : launch_grad_gemm<float2>(c, tau, n_tau, n_occ_tiles, n_vir_tiles);
        if (e != hipSuccess) return e;
    }
    if (grad_eps.any()) {
        eps_reduce_kernel<<<(c->nsp + 255) / 256, 256, 0, c->stream>>>(c->eps_part, n_rowtiles, c->nsp, grad_eps.out,
                                                                       grad_eps.sum, grad_eps.comp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_coef_grad(const mcmp2_ctx *c, grad_out grad_coeffs) {
    if (c->precision == MCMP2_BF16 || c->precision == MCMP2_FP16) return launch_coef_grad_lp(c, grad_coeffs);
    const double2 *psibar = reinterpret_cast<const double2 *>(c->psibar);
    const int n_tL = (c->nL + CGT - 1) / CGT, n_tS = (c->nS + CGT - 1) / CGT, n_tk = (c->nsp + CGT - 1) / CGT;
    const int n_items = (n_tL + n_tS) * n_tk;
    if (n_items >= 2 * c->n_cu) {  // 64 x 64 tiles once every CU gets two
        coef_grad_tile_kernel<<<8 * ((n_items + 7) / 8), 256, 0, c->stream>>>(
            c->XT, psibar, c->E, 2 * c->m, c->nb, c->nL, c->nsp, c->R, n_tL, n_tk, n_items,
            reinterpret_cast<double2 *>(grad_coeffs.out), reinterpret_cast<double2 *>(grad_coeffs.sum),
            reinterpret_cast<double2 *>(grad_coeffs.comp));
        return hipGetLastError();
    }
    {
        const int n_L_tiles = (c->nL + 15) / 16, n_S_tiles = (c->nS + 15) / 16;
        dim3 g2(n_L_tiles + n_S_tiles, (c->nsp + 15) / 16);
        coef_grad_kernel<<<g2, 256, 0, c->stream>>>(c->XT, psibar, c->E, 2 * c->m, c->nb, c->nL, c->nsp, c->R,
                                                    n_L_tiles, reinterpret_cast<double2 *>(grad_coeffs.out),
                                                    reinterpret_cast<double2 *>(grad_coeffs.sum),
                                                    reinterpret_cast<double2 *>(grad_coeffs.comp));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
