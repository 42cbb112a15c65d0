// HIP kernels of the LS-AMG-DD hot path for CDNA4 (gfx950).
//
// Setup: batched element eigendecompositions (element Gram factors, Sec. 5.2),
// assembly, batched local problems per aggregate (exact SPSD splitting,
// Schur complement, reduced generalized eigenproblem, mode selection,
// subdomain inverses; Sec. 2), Galerkin products G_T P_T (Sec. 2).
// Solve: CSR residuals, colour-parallel multiplicative Schwarz with
// explicit subdomain inverses, block-diagonal transfer, dense coarsest solve,
// PCG vector kernels.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "batched.hpp"
#include "dense.hpp"
#include "kernels.hpp"
#include "symv.hpp"

namespace lsdd {

// Kernel-bracketing timing events for the next subdomain-product launch (per host
// thread): the launch records them at the kernel's own start and end.
namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
}
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}
bool take_launch_events(hipEvent_t* start, hipEvent_t* stop) {
    if (!t_ev_start) return false;
    *start = t_ev_start;
    *stop = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    return true;
}

namespace {

constexpr int WG = LSDD_WG;
constexpr int NE_LDS = 48;          // element blocks up to this size stay in LDS

inline unsigned grid_for(int64_t n, int per_block = WG) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65535LL * 64) g = 65535LL * 64;
    return (unsigned)g;
}

__device__ inline int64_t find_slot(const int32_t* col, int64_t lo, int64_t hi, int32_t q) {
    // binary search for column q in col[lo, hi)
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t c = col[mid];
        if (c < q) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// position of DOF q inside Omega = [omega ascending | Gamma ascending], or -1
__device__ inline int local_index(const int32_t* dofs, int nw, int m, int32_t q) {
    int lo = 0, hi = nw;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (dofs[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    if (lo < nw && dofs[lo] == q) return lo;
    lo = nw;
    hi = m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (dofs[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    if (lo < m && dofs[lo] == q) return lo;
    return -1;
}

// ====================================================================== K1: element Gram factors

// One workgroup per element: eigendecomposition of the symmetric block A_T by
// parallel Jacobi, SPSD check, rank, and G_T = Lambda_+^{1/2} Q_+^T stored
// row-major as an n_T x n_T array whose first r_T rows are valid.  Blocks up to
// NE_LDS: the rotated matrix and the eigenvectors live in dynamic LDS (lds_bytes,
// sized to the largest block so small blocks leave room for many workgroups per
// CU), the sorted vectors in the element's slot of scratch; larger blocks are
// left to k_elem_eig_trd.
__global__ void __launch_bounds__(WG) k_elem_eig(const int64_t* elem_ptr, const int64_t* blk_off,
                                                 const double* blocks, double* G, int32_t* ranks,
                                                 int32_t* status, double* scratch, int64_t scratch_stride,
                                                 double rank_rtol, double spsd_tol, int64_t lds_bytes) {
    extern __shared__ double s_dyn[];
    __shared__ double s_w[128];
    __shared__ int s_rank[128];
    __shared__ int s_pairs[128];
    __shared__ double s_cs[128];
    __shared__ int s_flag;
    __shared__ double s_red[WG / 64];
    const int64_t e = blockIdx.x;
    const int n = (int)(elem_ptr[e + 1] - elem_ptr[e]);
    const double* B = blocks + blk_off[e];
    if (n > NE_LDS) return;                   // k_elem_eig_trd
    const int64_t nn = (int64_t)n * n;
    double* a = s_dyn;                         // lds_bytes >= 2 n^2 doubles
    double* v = s_dyn + nn;
    double* vs = scratch + e * scratch_stride; // sorted vectors (global, n^2)
    // load (column-major == row-major for symmetric), asymmetry and scale
    double asym = 0.0, amax = 0.0;
    for (int idx = tid(); idx < n * n; idx += WG) {
        int i = idx % n, j = idx / n;
        double x = B[(int64_t)i * n + j], y = B[(int64_t)j * n + i];
        a[i + j * n] = 0.5 * (x + y);
        asym = fmax(asym, fabs(x - y));
        amax = fmax(amax, fabs(x));
    }
    __syncthreads();
    asym = wg_max(asym, s_red);
    amax = wg_max(amax, s_red);
    if (!(asym <= 1e-12 * amax) || !(amax == amax) || amax > DBL_MAX) {
        if (tid() == 0) status[e] = 1;   // asymmetric or non-finite
        return;
    }
    wg_identity(v, n, n);
    wg_jacobi(a, n, n, v, n, 60, 1e-15, 1e-18 * amax, s_pairs, s_cs, &s_flag);
    wg_sort_eig(a, n, v, n, n, s_w, vs, n, s_rank);
    const double lmax = fmax(s_w[n - 1], 0.0);
    if (s_w[0] < -spsd_tol * lmax) {
        if (tid() == 0) status[e] = 2;
        return;
    }
    const double tol = (rank_rtol > 0.0 ? rank_rtol : n * DBL_EPSILON) * lmax;
    int first = 0;
    while (first < n && !(s_w[first] > tol)) ++first;   // eigenvalues ascending
    const int r = n - first;
    double* g = G + blk_off[e];
    for (int idx = tid(); idx < n * n; idx += WG) {
        int row = idx / n, c = idx % n;
        double val = 0.0;
        if (row < r) {
            int t = first + row;
            val = sqrt(s_w[t]) * vs[c + (int64_t)t * n];
        }
        g[idx] = val;
    }
    if (tid() == 0) {
        ranks[e] = r;
        status[e] = 0;
    }
}

// Element blocks larger than NE_LDS, one workgroup per element: the same outputs
// and rules as k_elem_eig (SPSD check, rank at n_T eps lambda_max, G_T =
// Lambda_+^{1/2} Q_+^T with rows in ascending eigenvalue order) from a Householder
// tridiagonalisation, bisection for all eigenvalues, inverse iteration for the
// retained ones only and back-transformation, instead of Jacobi sweeps.  Four
// launches (PHASE 0..3: load and reduce; eigenvalues, SPSD check and rank;
// inverse iteration; back-transformation and G_T), so that the register-heavy
// inverse iteration does not set the occupancy of the others.  The element's slot
// of scratch holds S (n^2, reduced in place) | V (n^2, retained vectors) | d, e,
// tau, w (4n) | inverse-iteration scratch (INVIT_SLOTS n + 4096); status[e] and
// ranks[e] carry the state between phases.  Dynamic LDS: 2 n_max + 64 doubles.
// Smaller elements are left to k_elem_eig.
template <int PHASE>
__global__ void __launch_bounds__(WG) k_elem_eig_trd(const int64_t* elem_ptr, const int64_t* blk_off,
                                                     const double* blocks, double* G, int32_t* ranks,
                                                     int32_t* status, double* scratch, int64_t scratch_stride,
                                                     double rank_rtol, double spsd_tol) {
    extern __shared__ double s_dyn[];
    __shared__ double s_red[WG / 64];
    __shared__ int s_ncl;
    const int64_t e = blockIdx.x;
    const int n = (int)(elem_ptr[e + 1] - elem_ptr[e]);
    if (n <= NE_LDS) return;
    if (PHASE > 0 && status[e] != 0) return;
    const int64_t nn = (int64_t)n * n;
    double* S = scratch + e * scratch_stride;
    double* V = S + nn;
    double* d = V + nn;
    double* ee = d + n;
    double* tau = ee + n;
    double* w = tau + n;
    double* ws = w + n;
    if (PHASE == 0) {
        const double* B = blocks + blk_off[e];
        double asym = 0.0, amax = 0.0;
        for (int idx = tid(); idx < n * n; idx += WG) {
            const int i = idx % n, j = idx / n;
            const double x = B[(int64_t)i * n + j], y = B[(int64_t)j * n + i];
            S[i + (int64_t)j * n] = 0.5 * (x + y);
            asym = fmax(asym, fabs(x - y));
            amax = fmax(amax, fabs(x));
        }
        __syncthreads();
        asym = wg_max(asym, s_red);
        amax = wg_max(amax, s_red);
        if (!(asym <= 1e-12 * amax) || !(amax == amax) || amax > DBL_MAX) {
            if (tid() == 0) status[e] = 1;   // asymmetric or non-finite
            return;
        }
        wg_tridiag(S, n, d, ee, tau, s_dyn, s_dyn + n, s_red);
        if (tid() == 0) status[e] = 0;
        return;
    }
    if (PHASE == 1) {
        wg_bisect_all(d, ee, n, w, s_red);
        __syncthreads();
        if (tid() == 0) {
            const double lmax = fmax(w[n - 1], 0.0);
            if (w[0] < -spsd_tol * lmax) {
                status[e] = 2;
            } else {
                const double tol = (rank_rtol > 0.0 ? rank_rtol : n * DBL_EPSILON) * lmax;
                int first = 0;
                while (first < n && !(w[first] > tol)) ++first;     // eigenvalues ascending
                ranks[e] = n - first;
            }
        }
        return;
    }
    const int r = ranks[e];
    const int first = n - r;
    if (PHASE == 2) {
        if (r == 0) return;
        double tnorm = 0.0;
        for (int i = tid(); i < n; i += WG)
            tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0));
        tnorm = wg_max(tnorm, s_red);
        wg_inverse_iteration(d, ee, n, w + first, r, V, ws, fmax(tnorm, 1e-300), (int*)s_dyn, s_dyn + n, s_red,
                             &s_ncl);
        return;
    }
    if (r > 0) wg_tridiag_backtransform(S, n, tau, V, r, s_dyn, s_dyn + n);
    double* g = G + blk_off[e];
    for (int idx = tid(); idx < n * n; idx += WG) {
        const int row = idx / n, c = idx % n;
        g[idx] = row < r ? sqrt(w[first + row]) * V[c + (int64_t)row * n] : 0.0;
    }
}

// One workgroup per element: pivoted Cholesky of the symmetric block A_T (Sec. 5.2,
// the direct alternative to the eigendecomposition).  Step k pivots on the largest
// remaining diagonal entry of the Schur complement S (lowest index among equal
// ones); row k of G_T is the pivot column of S scaled by 1/sqrt(pivot), zero on the
// DOFs already eliminated, and S loses its outer product.  The factorisation stops
// when the largest remaining diagonal entry is at most
// tol = (rank_rtol or n_T eps) max diag(A_T); the rank is the number of steps.  For
// an SPSD block the remainder is then bounded by tol entrywise, so a remainder
// entry above 2 max(tol, spsd_tol max diag), or a diagonal entry below
// -spsd_tol max diag, marks the block as not SPSD.  G_T is stored as by k_elem_eig.
__global__ void __launch_bounds__(WG) k_elem_pchol(const int64_t* elem_ptr, const int64_t* blk_off,
                                                   const double* blocks, double* G, int32_t* ranks,
                                                   int32_t* status, double* scratch, int64_t scratch_stride,
                                                   double rank_rtol, double spsd_tol) {
    __shared__ double s_a[NE_LDS * NE_LDS];
    __shared__ double s_g[128];
    __shared__ int s_live[128];
    __shared__ double s_red[WG / 64];
    const int64_t e = blockIdx.x;
    const int n = (int)(elem_ptr[e + 1] - elem_ptr[e]);
    const double* B = blocks + blk_off[e];
    double* a = n <= NE_LDS ? s_a : scratch + e * scratch_stride;
    double asym = 0.0, amax = 0.0, dmax = -DBL_MAX;
    for (int idx = tid(); idx < n * n; idx += WG) {
        int i = idx % n, j = idx / n;
        double x = B[(int64_t)i * n + j], y = B[(int64_t)j * n + i];
        a[i + j * n] = 0.5 * (x + y);
        asym = fmax(asym, fabs(x - y));
        amax = fmax(amax, fabs(x));
        if (i == j) dmax = fmax(dmax, x);
    }
    for (int i = tid(); i < n; i += WG) s_live[i] = 1;
    __syncthreads();
    asym = wg_max(asym, s_red);
    amax = wg_max(amax, s_red);
    dmax = wg_max(dmax, s_red);
    if (!(asym <= 1e-12 * amax) || !(amax == amax) || amax > DBL_MAX) {
        if (tid() == 0) status[e] = 1;   // asymmetric or non-finite
        return;
    }
    double* g = G + blk_off[e];
    if (!(dmax > 0.0)) {                 // zero block: rank 0; otherwise not SPSD
        for (int idx = tid(); idx < n * n; idx += WG) g[idx] = 0.0;
        if (tid() == 0) {
            ranks[e] = 0;
            status[e] = amax > 0.0 ? 2 : 0;
        }
        return;
    }
    const double tol = (rank_rtol > 0.0 ? rank_rtol : n * DBL_EPSILON) * dmax;
    int k = 0;
    for (; k < n; ++k) {
        double bv = -DBL_MAX;
        int bi = n;
        for (int i = tid(); i < n; i += WG) {
            const double d = a[i + (int64_t)i * n];
            if (s_live[i] && d > bv) {
                bv = d;
                bi = i;
            }
        }
        const double best = wg_max(bv, s_red);
        const int piv = (int)(-wg_max(-(double)(bv == best ? bi : n), s_red));   // lowest index of the maximum
        if (!(best > tol)) break;
        const double rs = 1.0 / sqrt(best);
        for (int i = tid(); i < n; i += WG) {
            const double v = s_live[i] ? a[i + (int64_t)piv * n] * rs : 0.0;
            s_g[i] = v;
            g[(int64_t)k * n + i] = v;
        }
        __syncthreads();
        for (int idx = tid(); idx < n * n; idx += WG) {
            const int i = idx % n, j = idx / n;
            if (s_live[i] && s_live[j]) a[idx] -= s_g[i] * s_g[j];
        }
        __syncthreads();
        if (tid() == 0) s_live[piv] = 0;
        __syncthreads();
    }
    for (int64_t idx = (int64_t)k * n + tid(); idx < (int64_t)n * n; idx += WG) g[idx] = 0.0;
    double rmax = 0.0, dneg = 0.0;
    for (int idx = tid(); idx < n * n; idx += WG) {
        const int i = idx % n, j = idx / n;
        if (s_live[i] && s_live[j]) {
            rmax = fmax(rmax, fabs(a[idx]));
            if (i == j) dneg = fmax(dneg, -a[idx]);
        }
    }
    rmax = wg_max(rmax, s_red);
    dneg = wg_max(dneg, s_red);
    const double chk = fmax(tol, spsd_tol * dmax);
    if (tid() == 0) {
        ranks[e] = k;
        status[e] = (dneg > spsd_tol * dmax || rmax > 2.0 * chk) ? 2 : 0;
    }
}

// ====================================================================== assembly into CSR

// Assembly A = sum_T R_T^T A_T R_T into a CSR pattern that contains every
// (p, q) of every support: one thread per row p visits the elements holding p
// in ascending order (deterministic summation order).
__global__ void k_assemble_rows(int64_t n, const int64_t* d2e_ptr, const int32_t* d2e_elem, const int32_t* d2e_loc,
                                const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* blk_off,
                                const double* blocks, const double* factor, const int64_t* rowptr, const int32_t* col,
                                double* val) {
    const int64_t p = blockIdx.x * (int64_t)WG + tid();
    if (p >= n) return;
    const int64_t lo = rowptr[p], hi = rowptr[p + 1];
    for (int64_t q = d2e_ptr[p]; q < d2e_ptr[p + 1]; ++q) {
        const int32_t e = d2e_elem[q];
        const int a = d2e_loc[q];
        const int64_t base = elem_ptr[e];
        const int ne = (int)(elem_ptr[e + 1] - base);
        const double* B = blocks + blk_off[e] + (int64_t)a * ne;
        const double f = factor ? factor[e] : 1.0;
        for (int b = 0; b < ne; ++b) {
            int64_t slot = find_slot(col, lo, hi, elem_dofs[base + b]);
            val[slot] += f * B[b];
        }
    }
}

// The same with one wave per row (for long element rows): lanes take the
// columns of an element, elements in the same order, so every entry receives
// its contributions in the same order as above.
__global__ void __launch_bounds__(WG) k_assemble_rows_wave(int64_t n, const int64_t* d2e_ptr,
                                                           const int32_t* d2e_elem, const int32_t* d2e_loc,
                                                           const int64_t* elem_ptr, const int32_t* elem_dofs,
                                                           const int64_t* blk_off, const double* blocks,
                                                           const double* factor, const int64_t* rowptr,
                                                           const int32_t* col, double* val) {
    const int lane = tid() & 63;
    const int64_t p = (blockIdx.x * (int64_t)WG + tid()) >> 6;
    if (p >= n) return;
    const int64_t lo = rowptr[p], hi = rowptr[p + 1];
    for (int64_t q = d2e_ptr[p]; q < d2e_ptr[p + 1]; ++q) {
        const int32_t e = d2e_elem[q];
        const int a = d2e_loc[q];
        const int64_t base = elem_ptr[e];
        const int ne = (int)(elem_ptr[e + 1] - base);
        const double* B = blocks + blk_off[e] + (int64_t)a * ne;
        const double f = factor ? factor[e] : 1.0;
        for (int b = lane; b < ne; b += 64) {
            const int64_t slot = find_slot(col, lo, hi, elem_dofs[base + b]);
            val[slot] += f * B[b];
        }
    }
}

// factor[e] = theta[e] / theta0[e] (theta0 NULL: theta[e])
__global__ void k_theta_factor(int64_t n, const double* theta, const double* theta0, double* factor) {
    for (int64_t e = blockIdx.x * (int64_t)WG + tid(); e < n; e += (int64_t)gridDim.x * WG)
        factor[e] = theta0 ? theta[e] / theta0[e] : theta[e];
}

// blocks of element e *= scale[e]
__global__ void k_scale_blocks(int64_t n_elem, const int64_t* blk_off, const double* scale, double* blocks) {
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const double s = scale[e];
        for (int64_t q = blk_off[e] + tid(); q < blk_off[e + 1]; q += WG) blocks[q] *= s;
    }
}

// Gram rows from diagonally pivoted Cholesky factors (Sec. 5.2).  Element e
// (n x n at blk_off[e]) holds in L the factor in pivot order (column-major, lower
// triangle: L(i, k) at i + k n), perm[i] (at perm_off[e] - perm_off[0]) is the
// index at pivot position i and rank[e] the number of pivots r.  Writes G_e
// row-major n x n with G_e(k, perm[i]) = L(i, k) for k < r, i >= k, zero
// elsewhere, so that G_e^T G_e = A_e up to the truncated remainder.
__global__ void k_gram_rows(int64_t n_elem, const int64_t* perm_off, const int64_t* blk_off, const double* L,
                            const int32_t* perm, const int32_t* rank, double* G) {
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const int n = (int)(perm_off[e + 1] - perm_off[e]);
        const int r = rank[e];
        const double* l = L + blk_off[e];
        const int32_t* pm = perm + (perm_off[e] - perm_off[0]);
        double* g = G + blk_off[e];
        for (int idx = tid(); idx < n * n; idx += WG) {
            const int k = idx / n, i = idx % n;
            g[(int64_t)k * n + pm[i]] = (k < r && i >= k) ? l[i + (int64_t)k * n] : 0.0;
        }
    }
}

// Element e of a black-box Gram factor is one row g of G with s stored entries
// (values at val + src_off[e]): G_e (s x s, row-major) holds g in its first row
// and zeros below, and the element block is A_e = g^T g.
__global__ void k_gram_csr_rows(int64_t n_elem, const int64_t* elem_ptr, const int64_t* src_off,
                                const int64_t* blk_off, const double* val, double* G, double* blocks) {
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const int s = (int)(elem_ptr[e + 1] - elem_ptr[e]);
        const double* g = val + src_off[e];
        double* ge = G + blk_off[e];
        double* be = blocks + blk_off[e];
        for (int idx = tid(); idx < s * s; idx += WG) {
            const int u = idx / s, v = idx % s;
            ge[idx] = u == 0 ? g[v] : 0.0;
            be[idx] = g[u] * g[v];
        }
    }
}

// out[e] = u_e^T B_e v_e (B_e row-major n_e x n_e at blk_off[e]); one wave per
// element: lane j sums u_i B_ij v_j over the rows i (coalesced row reads), then
// a fixed-order wave reduction.
__global__ void __launch_bounds__(WG) k_elem_bilinear(int64_t n_elem, const int64_t* elem_ptr,
                                                      const int32_t* elem_dofs, const int64_t* blk_off,
                                                      const double* blocks, const double* u, const double* v,
                                                      int32_t nrhs, int64_t ld, double scale, double* out) {
    const int lane = tid() & 63;
    const int64_t e = (int64_t)blockIdx.x * (WG / 64) + (tid() >> 6);
    if (e >= n_elem) return;
    const int64_t base = elem_ptr[e];
    const int ne = (int)(elem_ptr[e + 1] - base);
    const double* B = blocks + blk_off[e];
    double acc = 0.0;
    for (int32_t k = 0; k < nrhs; ++k) {
        const double* uk = u + (int64_t)k * ld;
        const double* vk = v + (int64_t)k * ld;
        for (int j = lane; j < ne; j += 64) {
            const double vj = vk[elem_dofs[base + j]];
            double t = 0.0;
            for (int i = 0; i < ne; ++i) t += uk[elem_dofs[base + i]] * B[(int64_t)i * ne + j];
            acc += t * vj;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) out[e] = scale * acc;
}

// ====================================================================== local problems

// Per aggregate: A~_Omega = sum_{T in cl(omega)} mult(T)^{-1} E_T^T A_T E_T
// (eq. SPSD_splitting under structural support) and A_Omega = A[Omega, Omega].
// Grid (column blocks, batch entries): workgroup x owns the Omega columns
// [x ASM_CW, (x + 1) ASM_CW) of both matrices, zeroes them and adds the closure
// elements in closure order (every entry is summed in the same order on every
// run; an element touches an entry at most once).  A_Omega is filled column by
// column from the CSR rows of the symmetric A_l.
constexpr int ASM_CW = 32;

__global__ void __launch_bounds__(WG) k_local_assemble(LocalArgs A) {
    __shared__ int s_cnt;
    __shared__ int s_j[ASM_CW];
    const int b = blockIdx.y;
    const int ag = A.agg_list ? A.agg_list[b] : A.first + b;
    const int64_t s0 = A.sub_ptr[ag];
    const int m = (int)(A.sub_ptr[ag + 1] - s0);
    const int c0 = (int)blockIdx.x * ASM_CW;
    if (c0 >= m) return;
    const int c1 = min(m, c0 + ASM_CW);
    const int nw = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    const int32_t* dofs = A.sub_dofs + s0;
    double* W1 = A.w1 + A.ws_off[b];
    double* W2 = A.w2 + A.ws_off[b];
    for (int64_t idx = tid(); idx < (int64_t)(c1 - c0) * m; idx += WG) {
        W1[(int64_t)c0 * m + idx] = 0.0;
        W2[(int64_t)c0 * m + idx] = 0.0;
    }
    __syncthreads();
    for (int64_t c = A.cl_ptr[ag]; c < A.cl_ptr[ag + 1]; ++c) {
        const int32_t e = A.cl_elems[c];
        const int ne = (int)(A.elem_ptr[e + 1] - A.elem_ptr[e]);
        const int32_t* pos = A.clpos + A.clpos_off[c];
        if (tid() == 0) s_cnt = 0;
        __syncthreads();
        for (int j = tid(); j < ne; j += WG) {
            const int pj = pos[j];
            if (pj >= c0 && pj < c1) s_j[atomicAdd(&s_cnt, 1)] = j;
        }
        __syncthreads();
        const int nj = s_cnt;
        if (nj > 0) {
            const double* Be = A.blocks + A.blk_off[e];
            const double w = 1.0 / (double)A.mult[e];
            for (int idx = tid(); idx < nj * ne; idx += WG) {
                const int i = idx % ne, j = s_j[idx / ne];
                const int pi = pos[i];   // < 0: outside an A-closure overlap
                if (pi >= 0) W1[pi + (int64_t)pos[j] * m] += w * Be[(int64_t)i * ne + j];
            }
        }
        __syncthreads();
    }
    // column a of A_Omega = row dofs[a] of A_l restricted to Omega; 8 threads per column
    for (int a = c0 + tid() / 8; a < c1; a += WG / 8) {
        const int32_t p = dofs[a];
        for (int64_t q = A.rowptr[p] + (tid() & 7); q < A.rowptr[p + 1]; q += 8) {
            const int li = local_index(dofs, nw, m, A.col[q]);
            if (li >= 0) W2[li + (int64_t)a * m] = A.val[q];
        }
    }
}

// Per aggregate: eigenpairs of C = L^{-1} S~ L^{-T} (held in the S buffer):
// Jacobi for small aggregates, otherwise Householder tridiagonalisation +
// bisection for all eigenvalues + inverse iteration for the retained vectors
// only; then the retained-mode count (eq. tau-cut with cluster completion).
// Writes mu (ascending, clamped at 0), k, and the first k eigenvectors of C into
// W1 (nw x k, ld nw).  Four launches (PHASE 0..3): reduction (or Jacobi),
// eigenvalues and mode count, inverse iteration, back-transformation; the state
// between them lives in the aggregate's global scratch.
template <int PHASE>
__global__ void __launch_bounds__(WG) k_local_eig(LocalArgs A) {
    __shared__ double s_red[WG / 64];
    __shared__ int s_flag;
    __shared__ int s_ncl;
    extern __shared__ double s_dyn[];
    const int b = blockIdx.x;
    const int ag = A.first + b;
    const int nw = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    double* W1 = A.w1 + A.ws_off[b];
    double* S = A.s_buf + A.sq_off[b];
    double* V = A.v_buf + A.sq_off[b];
    double* T = A.t_buf + A.t_off[b];
    double* mu = A.mu + A.mu_off[ag];
    double* VS = W1;
    const bool small = nw <= 32;
    if (PHASE == 0) {
        if (small) {
            int* pairs = (int*)s_dyn;
            double* cs = s_dyn + 32;
            int* rank = (int*)(s_dyn + 64);
            double scale = 0.0;
            for (int i = tid(); i < nw; i += WG) scale = fmax(scale, fabs(S[i + (int64_t)i * nw]));
            scale = wg_max(scale, s_red);
            wg_identity(V, nw, nw);
            wg_jacobi(S, nw, nw, V, nw, 60, 1e-15, 1e-18 * fmax(scale, 1e-300), pairs, cs, &s_flag);
            wg_sort_eig(S, nw, V, nw, nw, mu, VS, nw, rank);
        } else if (!(A.trd_min > 0 && nw >= A.trd_min)) {
            wg_tridiag(S, nw, T, T + nw, T + 2 * nw, s_dyn, s_dyn + nw, s_red);
        }
        return;
    }
    if (PHASE == 1) {
        if (!small && !(A.trd_min > 0 && nw >= A.trd_min)) wg_bisect_all(T, T + nw, nw, mu, s_red);
        for (int i = tid(); i < nw; i += WG) mu[i] = fmax(mu[i], 0.0);
        __syncthreads();
        if (tid() == 0) {
            int k;
            if (A.modes_fixed > 0) {
                k = A.modes_fixed < nw ? A.modes_fixed : nw;
            } else {
                k = 0;
                const double thr = A.thr_agg ? A.thr_agg[ag] : A.thr;
                while (k < nw && mu[k] < thr + A.band_tol) ++k;
            }
            while (k > 0 && k < nw && mu[k] - mu[k - 1] <= A.cluster_tol) ++k;
            A.k_out[ag] = k;
        }
        return;
    }
    const int k = A.k_out[ag];
    if (small || k == 0) return;
    if (PHASE == 2) {
        if (A.trd_min > 0 && nw >= A.trd_min) return;     // vectors by the multi-workgroup path
        const double* d = T;
        const double* e = T + nw;
        double tnorm = 0.0;
        for (int i = tid(); i < nw; i += WG)
            tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < nw ? fabs(e[i]) : 0.0));
        tnorm = wg_max(tnorm, s_red);
        wg_inverse_iteration(d, e, nw, mu, k, VS, T + 3 * nw, fmax(tnorm, 1e-300), (int*)s_dyn, s_dyn + nw, s_red,
                             &s_ncl);
        return;
    }
    if (A.trd_min > 0 && nw >= A.trd_min) return;     // back-transformed by the blocked path
    wg_tridiag_backtransform(S, nw, T + 2 * nw, VS, k, s_dyn, s_dyn + nw);
}

// Z_i staged row-major (nw x k) from the column-major vectors in W1.
__global__ void k_stage_z(LocalArgs A) {
    const int b = blockIdx.x;
    const int ag = A.first + b;
    const int nw = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    const int k = A.k_out[ag];
    const double* VS = A.w1 + A.ws_off[b];
    double* zs = A.zst + A.zst_off[ag];
    for (int idx = tid(); idx < nw * k; idx += WG) {
        int i = idx / k, s = idx % k;
        zs[idx] = VS[i + (int64_t)s * nw];
    }
}

// Small per-view helpers for the batched pipeline.
__global__ void k_views_max_diag(const double* base, const View* v, double* out) {
    __shared__ double red[WG / 64];
    const View x = v[blockIdx.x];
    double m = 0.0;
    for (int i = tid(); i < x.rows; i += WG) m = fmax(m, base[x.off + i + (int64_t)i * x.ld]);
    m = wg_max(m, red);
    if (tid() == 0) out[blockIdx.x] = m;
}
__global__ void k_views_add_diag(double* base, const View* v, const double* delta) {
    const View x = v[blockIdx.x];
    const double d = delta[blockIdx.x];
    for (int i = tid(); i < x.rows; i += WG) base[x.off + i + (int64_t)i * x.ld] += d;
}
__global__ void k_views_symmetrize(double* base, const View* v) {
    const View x = v[blockIdx.y];
    const int64_t n = x.rows;
    for (int64_t idx = (int64_t)blockIdx.x * WG + tid(); idx < n * n; idx += (int64_t)gridDim.x * WG) {
        int64_t i = idx % n, j = idx / n;
        if (i < j) {
            double s = 0.5 * (base[x.off + i + j * x.ld] + base[x.off + j + i * x.ld]);
            base[x.off + i + j * x.ld] = s;
            base[x.off + j + i * x.ld] = s;
        }
    }
}
__global__ void k_views_identity(double* base, const View* v) {
    const View x = v[blockIdx.y];
    const int64_t n = x.rows;
    for (int64_t idx = (int64_t)blockIdx.x * WG + tid(); idx < n * n; idx += (int64_t)gridDim.x * WG) {
        int64_t i = idx % n, j = idx / n;
        base[x.off + i + j * x.ld] = (i == j) ? 1.0 : 0.0;
    }
}

// Compact the staged Z_i (row-major) into Z (row-major, for the Galerkin
// products and export) and Zc / Zc32 (column-major, for the transfers).
__global__ void k_z_compact(const int64_t* agg_ptr, const int32_t* k, const int64_t* zst_off, const double* zst,
                            const int64_t* zoff, double* Z, double* Zc, float* Zc32) {
    const int ag = blockIdx.x;
    const int nw = (int)(agg_ptr[ag + 1] - agg_ptr[ag]);
    const int kk = k[ag];
    const int64_t cnt = (int64_t)nw * kk;
    const double* src = zst + zst_off[ag];
    for (int64_t i = tid(); i < cnt; i += WG) {
        double v = src[i];
        Z[zoff[ag] + i] = v;
        int64_t a = i / kk, s = i % kk;
        Zc[zoff[ag] + a + s * nw] = v;
        if (Zc32) Zc32[zoff[ag] + a + s * nw] = (float)v;
    }
}

// ====================================================================== Galerkin products

// Stacked interpolation rows of coarse group g = g0 + blockIdx.x: member e
// (in member order) contributes the n_e rows P_e = P[S_e, S_g], block
// structured by aggregate; column-major R_g x c_g with R_g = sum of n_e.
__global__ void __launch_bounds__(WG) k_build_pst(PstArgs g) {
    const int gi = g.g0 + (int)blockIdx.x;
    const int c = (int)(g.cptr[gi + 1] - g.cptr[gi]);
    const int64_t R = g.rows[blockIdx.x];
    double* P = g.pst + g.pst_off[blockIdx.x];
    int64_t row0 = 0;
    for (int64_t mi = g.mem_ptr[gi]; mi < g.mem_ptr[gi + 1]; ++mi) {
        const int32_t e = g.mem_elems[mi];
        const int ne = (int)(g.felem_ptr[e + 1] - g.felem_ptr[e]);
        const int64_t pm = g.pm_off[mi];
        for (int idx = tid(); idx < ne * c; idx += WG) {
            const int a = idx % ne, col = idx / ne;
            double v = 0.0;
            const int64_t zr = g.pm_zrow[pm + a];
            if (zr >= 0) {
                const int s = col - g.pm_col[pm + a];
                if (s >= 0 && s < g.pm_k[pm + a]) v = g.Z[zr + s];
            }
            P[row0 + a + (int64_t)col * R] = v;
        }
        row0 += ne;
    }
}

// ====================================================================== coarsest level

// D (n x n, column-major) = A[off:off+n, off:off+n]; entries outside the block are skipped
__global__ void k_dense_from_csr(int64_t off, int64_t n, const int64_t* rowptr, const int32_t* col,
                                 const double* val, double* D) {
    const int64_t p = blockIdx.x;
    for (int64_t q = rowptr[off + p] + tid(); q < rowptr[off + p + 1]; q += WG) {
        const int64_t c = (int64_t)col[q] - off;
        if (c >= 0 && c < n) D[p + c * n] = val[q];
    }
}


// ====================================================================== conversions

__global__ void k_to_f32(int64_t n, const double* a, float* b) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) b[i] = (float)a[i];
}
__global__ void k_to_f64(int64_t n, const float* a, double* b) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) b[i] = (double)a[i];
}

// ====================================================================== solve kernels

// out[t] = r[rows[t]] - sum_q A[rows[t], q] x[q]; L lanes per row (16 for
// short rows, a whole wave for the long rows of coarse levels).  The matrix
// streams (values, column indices) are read non-temporally, the gathered x
// through the caches.  Values of type V (FP64 values with FP32 vectors: the
// products and the sum are formed in FP64 and rounded once).
//
// scoff != NULL: the rows of a supernode share one column list (coarse levels,
// whose DOFs come in contiguous per-aggregate groups): row p's columns are
// col[scoff[p] ..] (read through the caches, reused by the supernode's other
// rows) and only the values stream, 8 bytes per entry instead of 12.
template <typename T, typename V, int L>
__global__ void __launch_bounds__(WG) k_csr_resid_rows(int64_t nrows, const int32_t* rows, const int64_t* rowptr,
                                                       const int32_t* col, const V* val, const T* x, const T* r,
                                                       T* out, int x_zero, const int64_t* scoff) {
    const int lane = tid() & (L - 1);
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t t = ((int64_t)blockIdx.x * WG + tid()) / L; t < nrows; t += stride) {
        const int32_t p = rows[t];   // < 0: masked entry, out = 0
        V s = 0;
        if (!x_zero && p >= 0) {
            // up to 4 entries per lane in flight: all column indices, then all
            // gathers, then the products (two dependent loads per entry).  The
            // loads carry no lane condition (a slot past the row's end re-reads its
            // last entry, same cache line, and contributes zero), so they are all
            // issued before the first wait.
            const int64_t qb = rowptr[p], q1 = rowptr[p + 1], qlast = q1 - 1;
            const int64_t cb = scoff ? scoff[p] - qb : 0;
            for (int64_t q0 = qb + lane; q0 < q1; q0 += 4 * L) {
                int32_t c[4];
                V v[4];
                T xv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = min(q0 + u * L, qlast);
                    c[u] = scoff ? col[cb + q] : __builtin_nontemporal_load(col + q);
                    v[u] = __builtin_nontemporal_load(val + q);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) xv[u] = x[c[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) s += (q0 + u * L < q1 ? v[u] : (V)0) * (V)xv[u];
            }
        }
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (lane == 0) out[t] = p >= 0 ? (T)((V)r[p] - s) : (T)0;
    }
}

// The residual rows of a supernode-blocked level by row blocks.  Block b is the run
// of list positions blk[2b] .. blk[2b] + blk[2b+1] - 1 (1 to 8 of them) whose rows
// belong to one supernode and so share one column list.  WPB waves of one workgroup
// per block split its column list in chunks of 128; per chunk a wave gathers x once
// and streams the (up to) 8 value rows against it, so the column indices and the
// gathered x cost one cache read per block instead of one per row.  A block of
// fewer than 8 rows repeats its last row in the spare slots (same addresses, never
// stored).  out[t] as in k_csr_resid_rows; every product and the per-lane sums as
// there, the cross-lane and cross-wave sums in another (fixed) order.
template <typename T, typename V, int WPB>
__global__ void __launch_bounds__(WG) k_sup_resid_blocks(int64_t nblk, const int32_t* blk, const int32_t* rows,
                                                         const int64_t* rowptr, const int32_t* scol,
                                                         const int64_t* scoff, const V* val, const T* x, const T* r,
                                                         T* out, int x_zero) {
    constexpr int RB = 8, U = 2, NW = WG / 64, BPW = NW / WPB;   // blocks per workgroup
    __shared__ V red[NW][RB];
    const int lane = tid() & 63, wave = tid() >> 6, wb = wave % WPB;
    const int j = (lane >> 3) & 7;   // the row whose sum lane j*8 ends with
    // the loop runs alike in every wave of the workgroup (barriers below)
    for (int64_t base = (int64_t)blockIdx.x * BPW; base < nblk; base += (int64_t)gridDim.x * BPW) {
        const int64_t b = base + wave / WPB;
        const bool act = b < nblk;
        int32_t t0 = 0, nb = 0;
        V a1 = 0;
        if (act) {
            t0 = blk[2 * b];
            nb = blk[2 * b + 1];
            const int32_t p0 = rows[t0];
            const int64_t qb = rowptr[p0], len = rowptr[p0 + 1] - qb;
            V s[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) s[i] = 0;
            if (!x_zero) {
                const V* vr[RB];
#pragma unroll
                for (int i = 0; i < RB; ++i) vr[i] = val + rowptr[rows[t0 + min(i, nb - 1)]];
                const int32_t* cl = scol + scoff[p0];
                for (int64_t q0 = lane + wb * U * 64; q0 < len; q0 += WPB * U * 64) {
                    int64_t qq[U];
                    int32_t c[U];
                    V v[RB][U];
                    T xv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        qq[u] = min(q0 + u * 64, len - 1);
                        c[u] = cl[qq[u]];
                    }
#pragma unroll
                    for (int i = 0; i < RB; ++i)
#pragma unroll
                        for (int u = 0; u < U; ++u) v[i][u] = __builtin_nontemporal_load(vr[i] + qq[u]);
#pragma unroll
                    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool in = q0 + u * 64 < len;
#pragma unroll
                        for (int i = 0; i < RB; ++i) s[i] += (in ? v[i][u] : (V)0) * (V)xv[u];
                    }
                }
            }
            // the 8 sums over the wave: exchanges over lane distances 32, 16, 8 halve
            // the rows each lane carries (lane l ends with row j over 8 lanes), then
            // distances 4, 2, 1 finish each row's sum
            const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
            V a4[4], a2[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) a4[i] = (h32 ? s[i + 4] : s[i]) + __shfl_xor(h32 ? s[i] : s[i + 4], 32);
#pragma unroll
            for (int i = 0; i < 2; ++i) a2[i] = (h16 ? a4[i + 2] : a4[i]) + __shfl_xor(h16 ? a4[i] : a4[i + 2], 16);
            a1 = (h8 ? a2[1] : a2[0]) + __shfl_xor(h8 ? a2[0] : a2[1], 8);
            a1 += __shfl_xor(a1, 4);
            a1 += __shfl_xor(a1, 2);
            a1 += __shfl_xor(a1, 1);
        }
        if constexpr (WPB > 1) {
            // the block's waves in order, summed by its first wave
            if ((lane & 7) == 0) red[wave][j] = a1;
            __syncthreads();
            if (wb == 0) {
#pragma unroll
                for (int w = 1; w < WPB; ++w) a1 += red[wave + w][j];
            }
            __syncthreads();
        }
        if (act && wb == 0 && (lane & 7) == 0 && j < nb) {
            const int32_t pj = rows[t0 + j];
            out[t0 + j] = (T)((V)r[pj] - a1);
        }
    }
}

// y = A x, or y = r_minus - A x when r_minus != nullptr (values of type V as in
// k_csr_resid_rows)
template <typename T, typename V, int L>
__global__ void __launch_bounds__(WG) k_csr_spmv(int64_t n, const int64_t* rowptr, const int32_t* col, const V* val,
                                                 const T* x, T* y, const T* r_minus, const int64_t* scoff) {
    const int lane = tid() & (L - 1);
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t p = ((int64_t)blockIdx.x * WG + tid()) / L; p < n; p += stride) {
        // as in k_csr_resid_rows: 4 entries per lane in flight, loads without lane
        // conditions (slots past the row's end re-read its last entry and add zero);
        // scoff != NULL: per-supernode column lists
        const int64_t qb = rowptr[p], q1 = rowptr[p + 1], qlast = q1 - 1;
        const int64_t cb = scoff ? scoff[p] - qb : 0;
        V s = 0;
        for (int64_t q0 = qb + lane; q0 < q1; q0 += 4 * L) {
            int32_t c[4];
            V v[4];
            T xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = min(q0 + u * L, qlast);
                c[u] = scoff ? col[cb + q] : __builtin_nontemporal_load(col + q);
                v[u] = __builtin_nontemporal_load(val + q);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) s += (q0 + u * L < q1 ? v[u] : (V)0) * (V)xv[u];
        }
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (lane == 0) y[p] = r_minus ? (T)((V)r_minus[p] - s) : (T)s;
    }
}

// Element-batch operator apply (Sec. 2, A = sum_T R_T^T A_T R_T with A_T = G_T^T G_T):
// ybuf[elem_ptr[e] + j] = (A_e x_e)_j from the packed lower triangle of A_e (row i
// at tri_off[e] + i (i + 1) / 2, entries A_e(i, 0 .. i)).  S lanes per element
// (S = 32: two elements per wave), C columns per lane (n_e <= S C).  Lane j forms
// y_j = sum_{i >= j} A_e(i, j) x_i by streaming the triangle row by row (row i is
// contiguous and read by lanes 0 .. i, coalesced), then adds sum_{k < j} A_e(j, k)
// x_k from its own row, which the first pass has just brought into the caches.
// Fixed order: ascending i, then ascending k.  Values of type V, vectors of type T
// (FP64 entries with FP32 vectors: FP64 sums, ybuf in FP64).
template <typename T, typename V, int S, int C>
__global__ void __launch_bounds__(WG) k_elem_tri_apply(int64_t n_elem, const int64_t* elem_ptr,
                                                       const int32_t* elem_dofs, const int64_t* tri_off,
                                                       const V* tri, const T* x, V* ybuf) {
    constexpr int SL = WG / S;
    __shared__ V s_x[SL][S * C];
    const int slot = tid() / S, lane = tid() % S;
    for (int64_t e0 = (int64_t)blockIdx.x * SL; e0 < n_elem; e0 += (int64_t)gridDim.x * SL) {
        const int64_t e = e0 + slot;
        const bool on = e < n_elem;
        const int64_t a0 = on ? elem_ptr[e] : 0;
        const int n = on ? (int)(elem_ptr[e + 1] - a0) : 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = lane + S * c;
            if (j < n) s_x[slot][j] = (V)x[elem_dofs[a0 + j]];
        }
        __syncthreads();
        V y[C];
#pragma unroll
        for (int c = 0; c < C; ++c) y[c] = 0;
        if (on) {
            // eight rows (pass 1) or entries (pass 2) per step, all loads issued before
            // the first use: the indices are clamped into the triangle instead of the
            // loads being conditional, and the clamped slots contribute nothing
            const V* t0 = tri + tri_off[e];
            for (int i0 = 0; i0 < n; i0 += 8) {
                V a[8][C];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = min(i0 + q, n - 1);
                    const V* row = t0 + (int64_t)i * (i + 1) / 2;
#pragma unroll
                    for (int c = 0; c < C; ++c) a[q][c] = row[min(lane + S * c, i)];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = i0 + q;
                    if (i < n) {
                        const V xi = s_x[slot][i];
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            if (lane + S * c <= i) y[c] += a[q][c] * xi;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int j = lane + S * c;
                if (j < n) {
                    const V* row = t0 + (int64_t)j * (j + 1) / 2;
                    V u = y[c];
                    for (int k0 = 0; k0 < j; k0 += 8) {
                        V a[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) a[q] = row[min(k0 + q, j - 1)];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (k0 + q < j) u += a[q] * s_x[slot][k0 + q];
                    }
                    ybuf[a0 + j] = u;
                }
            }
        }
        __syncthreads();
    }
}

// y[d] = sum over the elements holding DOF d (ascending) of their ybuf entries, or
// r_minus[d] minus that sum.
template <typename T, typename V>
__global__ void k_elem_gather(int64_t n, const int64_t* d2e_ptr, const int32_t* e2y, const V* ybuf,
                              const T* r_minus, T* y) {
    for (int64_t d = blockIdx.x * (int64_t)WG + tid(); d < n; d += (int64_t)gridDim.x * WG) {
        const int64_t q0 = d2e_ptr[d], q1 = d2e_ptr[d + 1];
        V s = 0;
        for (int64_t q = q0; q < q1; ++q) s += ybuf[e2y[q]];
        y[d] = r_minus ? (T)((V)r_minus[d] - s) : (T)s;
    }
}

// Packed lower triangles of factor[e] * A_e (factor NULL: 1) from the row-major
// blocks, in FP64 and (tri32 != NULL) FP32.
__global__ void k_pack_elem_tri(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                                const double* factor, const int64_t* tri_off, double* tri, float* tri32) {
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const int n = (int)(elem_ptr[e + 1] - elem_ptr[e]);
        const double f = factor ? factor[e] : 1.0;
        const double* B = blocks + blk_off[e];
        for (int idx = tid(); idx < n * (n + 1) / 2; idx += WG) {
            int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > idx) --i;
            while ((i + 1) * (i + 2) / 2 <= idx) ++i;
            const int j = idx - i * (i + 1) / 2;
            const double v = f * B[(int64_t)i * n + j];
            tri[tri_off[e] + idx] = v;
            if (tri32) tri32[tri_off[e] + idx] = (float)v;
        }
    }
}

// Subdomain correction with the packed symmetric inverse: A_Omega^{-1} is stored
// as its lower 64 x 64 tiles (tile (I, J), I >= J, row-major inside the tile,
// zero-padded past |Omega|; the diagonal tiles hold both triangles, of which
// only the lower one is read).  Work item = (subdomain, tile row I, chunk of up
// to `chl` tiles J): waves split the 64 rows of the tile row, lanes the 64
// columns.  Tile (I, J) is read once and used twice: its rows give
// y_I += T x_J (per-lane partials, reduced across lanes once per item) and its
// columns give y_J += T^T x_I (J < I; kept in registers and summed over the
// waves in LDS once per item); on the diagonal tile the columns of the strict
// lower triangle give the upper part of the product and are added to the
// item's row part.  Partial results go to a per-subdomain scratch -- row parts
// per (tile row, chunk), column parts per tile -- that k_sub_finalize sums in a
// fixed order, so the smoother is the same linear map on every application (no
// order-dependent atomics).
template <typename T>
__global__ void __launch_bounds__(WG) k_sub_symv(const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                                                 const T* tiles, const T* rloc, const int64_t* scr_off, T* scr,
                                                 int chl) {
    __shared__ T s_x[SUB_MAX_CHUNK * 64];
    __shared__ T s_xi[64];
    __shared__ T s_c[4][SUB_MAX_CHUNK][64];
    __shared__ T s_d[4][64];
    const int s = items[3 * blockIdx.x];
    const int I = items[3 * blockIdx.x + 1];
    const int ch = items[3 * blockIdx.x + 2];
    const int64_t o = sub_off[s];
    const int m = (int)(sub_off[s + 1] - o);
    const int nt = (m + 63) >> 6;
    const int J0 = ch * chl;
    const int nJ = min(chl, I + 1 - J0);       // tiles J0 .. J0 + nJ - 1
    const int ncol = min(nJ, I - J0);          // of which strictly below the diagonal
    for (int a = tid(); a < nJ * 64; a += WG) {
        int c = J0 * 64 + a;
        s_x[a] = c < m ? rloc[o + c] : (T)0;
    }
    const int lane = tid() & 63, w = tid() >> 6;
    if (tid() < 64) {
        const int r = I * 64 + tid();
        s_xi[tid()] = r < m ? rloc[o + r] : (T)0;
    }
    __syncthreads();
    const T* row0 = tiles + tp_off[s] + (int64_t)I * (I + 1) / 2 * 4096;
    T* part = scr + scr_off[s];
    T* colpart = part + symv_rowpart_off(nt, chl) * 64;
    T p[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) p[q] = 0;
    // Tiles are streamed once per application (non-temporal loads), two register
    // buffers deep: the loads of tile jj + 1 are in flight while tile jj is used.
    // The loads carry no lane condition: on the diagonal tile a lane above the
    // diagonal reads the row's diagonal entry instead (a cache line the row's
    // lower part fetches anyway) and its value is zeroed afterwards.
    T va[16], vb[16];
    auto fetch = [&](T(&v)[16], int jj) {
        const bool dg = J0 + jj == I;
        const T* t = row0 + (int64_t)(J0 + jj) * 4096;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = w + 4 * q;
            v[q] = __builtin_nontemporal_load(t + r * 64 + (dg ? min(lane, r) : lane));
        }
    };
    auto use = [&](const T(&v)[16], int jj) {
        const bool dg = J0 + jj == I;
        const T xj = s_x[jj * 64 + lane];
        T col = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = w + 4 * q;
            const T a = (dg && lane > r) ? (T)0 : v[q];
            p[q] += a * xj;
            col += ((dg && lane == r) ? (T)0 : a) * s_xi[r];
        }
        if (dg) s_d[w][lane] = col;
        else s_c[w][jj][lane] = col;
    };
    fetch(va, 0);
#pragma unroll
    for (int jj = 0; jj < SUB_MAX_CHUNK; jj += 2) {
        if (jj < nJ) {
            if (jj + 1 < nJ) fetch(vb, jj + 1);
            use(va, jj);
        }
        if (jj + 1 < nJ) {
            if (jj + 2 < nJ) fetch(va, jj + 2);
            use(vb, jj + 1);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        T v = p[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        p[q] = v;
    }
    __syncthreads();
    if (lane < 16) {
        T y = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (q == lane) y = p[q];
        const int r = w + 4 * lane;
        if (ncol < nJ) y += (s_d[0][r] + s_d[1][r]) + (s_d[2][r] + s_d[3][r]);
        part[(symv_rowpart_off(I, chl) + ch) * 64 + r] = y;
    }
    for (int a = tid(); a < ncol * 64; a += WG) {
        const int jj = a >> 6, l = a & 63;
        colpart[((int64_t)I * (I - 1) / 2 + J0 + jj) * 64 + l] =
            (s_c[0][jj][l] + s_c[1][jj][l]) + (s_c[2][jj][l] + s_c[3][jj][l]);
    }
}

// Factor-form local solve y = X^T (X r) of the mixed cycle in one pass over the
// FP32 factor tiles (the lower tiles of X = L^{-1} in the storage of k_sub_symv,
// zero above the diagonal), FP64 sums.  Work item = (subdomain, whole tile row
// I).  Phase 1 streams the row's tiles through the caches and forms
// w_I = sum_{J <= I} X_IJ r_J (waves split the 64 rows, lanes the 64 columns,
// per-lane partial sums reduced across the lanes once per item).  Phase 2 reads
// the same tiles again, now from the caches, with the same lane mapping: each
// wave forms the products of its 16 rows of w_I with the tile's columns and the
// four waves' partials are added in LDS: X_IJ^T w_I is the column part of tile (I, J);
// the diagonal tile's goes to the row-part slot of the chunk that holds it and
// the row's other chunk slots get zero, so k_sub_finalize sums the same layout as
// for the symmetric product.  HBM reads one pass of X (half the bytes of the FP64
// inverse) instead of two.
//
// stash > 0: the first `stash` tiles of the row also go to LDS (dynamic shared
// memory, stash * 16 KB) in phase 1, and phase 2 takes them from there; every
// thread reads back exactly the entries it stored, so no barrier separates the
// phases.  Tiles past `stash` are read again through the caches.
__global__ void __launch_bounds__(WG) k_sub_fact(const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                                                 const float* tiles, const float* rloc, const int64_t* scr_off,
                                                 float* scr, int chl, int stash) {
    constexpr int CH = 8;                                   // tiles per phase-2 LDS round
    extern __shared__ float s_stash[];
    __shared__ double s_c[4][CH][64];
    const int s = items[2 * blockIdx.x];
    const int I = items[2 * blockIdx.x + 1];
    const int64_t o = sub_off[s];
    const int m = (int)(sub_off[s + 1] - o);
    const int nt = (m + 63) >> 6;
    const int lane = tid() & 63, w = tid() >> 6;
    const float* row0 = tiles + tp_off[s] + (int64_t)I * (I + 1) / 2 * 4096;
    float* part = scr + scr_off[s];
    float* colpart = part + symv_rowpart_off(nt, chl) * 64;
    double p[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) p[q] = 0.0;
    float va[16], vb[16];
    // waves split the tile's 64 rows (row w + 4 q), lanes its columns
    auto fetch = [&](float(&v)[16], int J) {
        const float* t = row0 + (int64_t)J * 4096;
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = t[(w + 4 * q) * 64 + lane];
    };
    // phase 1: per-lane partials of w_I = sum_J X_IJ r_J
    auto use1 = [&](const float(&v)[16], int J) {
        const int c = J * 64 + lane;
        const double xj = c < m ? (double)rloc[o + c] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) p[q] += (double)v[q] * xj;
        if (J < stash)
#pragma unroll
            for (int q = 0; q < 16; ++q) s_stash[J * 4096 + (w + 4 * q) * 64 + lane] = v[q];
    };
    auto fetch2 = [&](float(&v)[16], int J) {
        if (J < stash) {
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = s_stash[J * 4096 + (w + 4 * q) * 64 + lane];
        } else {
            fetch(v, J);
        }
    };
    fetch(va, 0);
    for (int J = 0; J <= I; J += 2) {
        if (J + 1 <= I) fetch(vb, J + 1);
        use1(va, J);
        if (J + 1 <= I) {
            if (J + 2 <= I) fetch(va, J + 2);
            use1(vb, J + 1);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double v = p[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        p[q] = v;                                           // w_I[w + 4 q], on every lane
    }
    // phase 2: column parts X_IJ^T w_I, the row's tiles read again (now from the
    // caches) in rounds of CH tiles; per-wave partials summed over the waves in LDS
    auto use2 = [&](const float(&v)[16], int jj) {
        double col = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) col += (double)v[q] * p[q];
        s_c[w][jj][lane] = col;
    };
    for (int J0 = 0; J0 <= I; J0 += CH) {
        const int nJ = min(CH, I + 1 - J0);
        fetch2(va, J0);
#pragma unroll
        for (int jj = 0; jj < CH; jj += 2) {
            if (jj < nJ) {
                if (jj + 1 < nJ) fetch2(vb, J0 + jj + 1);
                use2(va, jj);
            }
            if (jj + 1 < nJ) {
                if (jj + 2 < nJ) fetch2(va, J0 + jj + 2);
                use2(vb, jj + 1);
            }
        }
        __syncthreads();
        for (int a = tid(); a < nJ * 64; a += WG) {
            const int jj = a >> 6, l = a & 63, J = J0 + jj;
            const float v = (float)((s_c[0][jj][l] + s_c[1][jj][l]) + (s_c[2][jj][l] + s_c[3][jj][l]));
            if (J < I) colpart[((int64_t)I * (I - 1) / 2 + J) * 64 + l] = v;
            else part[(symv_rowpart_off(I, chl) + I / chl) * 64 + l] = v;
        }
        __syncthreads();
    }
    if (w == 0)
        for (int ch = 0; ch < I / chl; ++ch) part[(symv_rowpart_off(I, chl) + ch) * 64 + lane] = 0.0f;
}

// x[Omega_s[c]] (+)= row-part chunks of tile row J(c) + column parts of the
// tile rows below.  FL threads per DOF each sum a fixed strided subset of the
// partials; the FL sums are added in LDS in ascending order (fixed order).
template <typename T, int FL>
__global__ void __launch_bounds__(WG) k_sub_finalize(int64_t r0, int64_t r1, const int32_t* pos_sub,
                                                     const int64_t* sub_off, const int64_t* scr_off, const T* scr,
                                                     const int32_t* sub_dofs, T* x, int accumulate, int chl) {
    constexpr int ND = WG / FL;
    __shared__ T s_y[FL][ND];
    const int dl = tid() % ND, j = tid() / ND;
    const int64_t t = r0 + (int64_t)blockIdx.x * ND + dl;
    T y = 0;
    if (t < r1) {
        const int s = pos_sub[t];
        const int64_t o = sub_off[s];
        const int c = (int)(t - o);
        const int nt = (int)((sub_off[s + 1] - o + 63) >> 6);
        const int J = c >> 6, l = c & 63;
        const T* part = scr + scr_off[s] + symv_rowpart_off(J, chl) * 64 + l;
        const T* colpart = scr + scr_off[s] + symv_rowpart_off(nt, chl) * 64 + l;
        const int nch = (J + chl) / chl;
        const int K = nch + (nt - 1 - J);
        // one load per partial, its address chosen without a branch so that the
        // unrolled loads are all in flight before the first wait
#pragma unroll 4
        for (int k = j; k < K; k += FL) {
            const int64_t I = J + 1 + (k - nch);
            y += *(k < nch ? part + (int64_t)k * 64 : colpart + (I * (I - 1) / 2 + J) * 64);
        }
    }
    s_y[j][dl] = y;
    __syncthreads();
    if (j == 0 && t < r1) {
        T v = s_y[0][dl];
#pragma unroll
        for (int q = 1; q < FL; ++q) v += s_y[q][dl];
        const int32_t d = sub_dofs ? sub_dofs[t] : (int32_t)t;   // < 0: masked entry
        if (d >= 0) x[d] = accumulate ? x[d] + v : v;
    }
}

// k_sub_finalize with the scratch addresses of every overlap entry precomputed
// (tab[t] = {row-part address of its first chunk, column-part address of tile row
// J's entry minus the tile-row offset, J, nch | nt << 16}, in scratch entries): the
// partial sums are one dependent load away from the table instead of three (entry ->
// subdomain -> offsets -> partials).  Same sums in the same order, accumulating.
template <typename T, int FL>
__global__ void __launch_bounds__(WG) k_sub_finalize_tab(int64_t r0, int64_t r1, const int4* tab, const T* scr,
                                                         const int32_t* sub_dofs, T* x) {
    constexpr int ND = WG / FL;
    __shared__ T s_y[FL][ND];
    const int dl = tid() % ND, j = tid() / ND;
    const int64_t t = r0 + (int64_t)blockIdx.x * ND + dl;
    T y = 0;
    if (t < r1) {
        const int4 e = tab[t];
        const T* part = scr + (uint32_t)e.x;
        const T* colpart = scr + (uint32_t)e.y;
        const int J = e.z, nch = e.w & 0xffff, nt = e.w >> 16;
        const int K = nch + (nt - 1 - J);
#pragma unroll 4
        for (int k = j; k < K; k += FL) {
            const int64_t I = J + 1 + (k - nch);
            y += *(k < nch ? part + (int64_t)k * 64 : colpart + I * (I - 1) / 2 * 64);
        }
    }
    s_y[j][dl] = y;
    __syncthreads();
    if (j == 0 && t < r1) {
        T v = s_y[0][dl];
#pragma unroll
        for (int q = 1; q < FL; ++q) v += s_y[q][dl];
        const int32_t d = sub_dofs[t];   // < 0: masked entry
        if (d >= 0) x[d] = x[d] + v;
    }
}

// Pack full m x m symmetric inverses (aggregate order, column-major) into the
// tiled lower storage of k_sub_symv (FP64 and, optionally, FP32).
__global__ void k_pack_tiles(const int64_t* sub_ptr, const int64_t* inv_off, const double* inv, const int64_t* tp_off,
                             double* tiles, float* tiles32) {
    const int ag = blockIdx.y;
    if (tp_off[ag] < 0) return;                   // stored in the small (packed) format
    const int m = (int)(sub_ptr[ag + 1] - sub_ptr[ag]);
    const int nt = (m + 63) / 64;
    const int64_t ntile = (int64_t)nt * (nt + 1) / 2;
    const double* M = inv + inv_off[ag];
    for (int64_t idx = (int64_t)blockIdx.x * WG + tid(); idx < ntile * 4096; idx += (int64_t)gridDim.x * WG) {
        int64_t t = idx >> 12;
        int e = (int)(idx & 4095);
        int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)I * (I + 1) / 2 > t) --I;
        while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
        int J = (int)(t - (int64_t)I * (I + 1) / 2);
        int r = I * 64 + (e >> 6), c = J * 64 + (e & 63);
        double v = (r < m && c < m) ? M[r + (int64_t)c * m] : 0.0;
        if (tiles) tiles[tp_off[ag] + idx] = v;
        if (tiles32) tiles32[tp_off[ag] + idx] = (float)v;
    }
}

// Packed lower triangles of the inverses of the aggregates with pk_off[a] >= 0
// (row-major packed: entry (i, j), j <= i, at i (i + 1) / 2 + j).
__global__ void k_pack_small(const int64_t* sub_ptr, const int64_t* inv_off, const double* inv,
                             const int64_t* pk_off, double* pk, float* pk32) {
    const int ag = blockIdx.x;
    if (pk_off[ag] < 0) return;
    const int m = (int)(sub_ptr[ag + 1] - sub_ptr[ag]);
    const double* M = inv + inv_off[ag];
    for (int e = tid(); e < m * (m + 1) / 2; e += WG) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (i * (i + 1) / 2 > e) --i;
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        const int j = e - i * (i + 1) / 2;
        const double v = M[i + (int64_t)j * m];
        if (pk) pk[pk_off[ag] + e] = v;
        if (pk32) pk32[pk_off[ag] + e] = (float)v;
    }
}

// Transfers with Z_i stored column-major (|omega_i| x k_i, column s contiguous).
// Restriction rc[coff_i + s] = sum_a Z_i[a, s] t[omega_i[a]]: work item =
// (aggregate, 16 columns); t on omega_i is staged in LDS in chunks of 2048
// rows, each wave takes 4 columns and its lanes stride the rows (coalesced),
// then a wave reduction per column.
template <typename T>
__global__ void __launch_bounds__(WG) k_restrict(const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                                                 const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc,
                                                 const T* t, T* rc) {
    __shared__ T s_t[2048];
    const int ag = items[2 * blockIdx.x], s0 = items[2 * blockIdx.x + 1];
    const int kk = k[ag];
    const int64_t a0 = agg_ptr[ag];
    const int nw = (int)(agg_ptr[ag + 1] - a0);
    const int lane = tid() & 63, w = tid() >> 6;
    const T* z = Zc + zoff[ag];
    T acc[4] = {0, 0, 0, 0};
    for (int c0 = 0; c0 < nw; c0 += 2048) {
        const int cn = min(2048, nw - c0);
        __syncthreads();
        // gather t over the chunk: all index loads, then all value loads (slots past the
        // chunk re-read its last entry and are not stored), so the two dependent loads
        // are paid once per four entries instead of once per entry
        for (int b = tid(); b < cn; b += 4 * WG) {
            int32_t d[4];
            T tv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u] = agg_dofs[a0 + c0 + min(b + u * WG, cn - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) tv[u] = t[d[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (b + u * WG < cn) s_t[b + u * WG] = tv[u];
        }
        __syncthreads();
        // the wave's 4 columns x 4 rows per lane in flight at once; out-of-range
        // columns and rows re-read an in-range entry and contribute zero
        const T* col[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) col[i] = z + (int64_t)min(s0 + w + 4 * i, kk - 1) * nw + c0;
        for (int a = lane; a < cn; a += 256) {
            T zv[4][4], tv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int aa = min(a + 64 * u, cn - 1);
                tv[u] = (a + 64 * u < cn) ? s_t[aa] : (T)0;
#pragma unroll
                for (int i = 0; i < 4; ++i) zv[i][u] = col[i][aa];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[i] += zv[i][u] * tv[u];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int s = s0 + w + 4 * i;
        T v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0 && s < kk) rc[coff[ag] + s] = v;
    }
}

// Prolongation x[omega_i[a]] += sum_s Z_i[a, s] ec[coff_i + s]: work item =
// (aggregate, 256 rows); thread per row, coalesced over rows, ec staged in LDS
// in chunks of 2048 modes.
template <typename T>
__global__ void __launch_bounds__(WG) k_prolong(const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                                                const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc,
                                                const T* ec, T* x) {
    __shared__ T s_e[2048];
    const int ag = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
    const int kk = k[ag];
    const int64_t a0 = agg_ptr[ag];
    const int nw = (int)(agg_ptr[ag + 1] - a0);
    const int a = r0 + tid();
    const T* z = Zc + zoff[ag] + a;
    T acc0 = 0, acc1 = 0;
    for (int c0 = 0; c0 < kk; c0 += 2048) {
        const int cn = min(2048, kk - c0);
        __syncthreads();
        for (int s = tid(); s < cn; s += WG) s_e[s] = ec[coff[ag] + c0 + s];
        __syncthreads();
        if (a < nw) {
            // PU modes per step in flight; modes past the end re-read the last one
            // and contribute zero
            constexpr int PU = 8;
            for (int s = 0; s < cn; s += PU) {
                T zv[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) zv[u] = z[(int64_t)(c0 + min(s + u, cn - 1)) * nw];
#pragma unroll
                for (int u = 0; u < PU; ++u) (u & 1 ? acc1 : acc0) += (s + u < cn ? zv[u] : (T)0) * s_e[min(s + u, cn - 1)];
            }
        }
    }
    if (a < nw) x[agg_dofs[a0 + a]] += acc0 + acc1;
}

template <typename T>
__global__ void k_zero(int64_t n, T* x) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) x[i] = 0;
}

// ---------------------------------------------------------------- PCG helpers

__global__ void __launch_bounds__(WG) k_dot_partial(int64_t n, const double* a, const double* b, double* partials) {
    __shared__ double red[WG / 64];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) s += a[i] * b[i];
    s = wg_sum(s, red);
    if (tid() == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(WG) k_sum_partials(int np, const double* partials, double* out) {
    __shared__ double red[WG / 64];
    double s = 0.0;
    for (int i = tid(); i < np; i += WG) s += partials[i];
    s = wg_sum(s, red);
    if (tid() == 0) *out = s;
}

__global__ void __launch_bounds__(WG) k_update_xr(int64_t n, const double* s_num, const double* s_den, const double* p,
                                                  const double* q, double* x, double* r, double* partials) {
    __shared__ double red[WG / 64];
    const double alpha = *s_num / *s_den;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = wg_sum(s, red);
    if (tid() == 0) partials[blockIdx.x] = s;
}

__global__ void k_update_p(int64_t n, const double* s_num, const double* s_den, const double* z, double* p) {
    const double beta = *s_num / *s_den;
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) p[i] = z[i] + beta * p[i];
}

__global__ void k_copy(int64_t n, const double* a, double* b) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) b[i] = a[i];
}

__global__ void k_axpy(int64_t n, double a, const double* x, double* y) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG) y[i] += a * x[i];
}

__global__ void k_check_finite(int64_t n, const double* a, int32_t* flag) {
    for (int64_t i = blockIdx.x * (int64_t)WG + tid(); i < n; i += (int64_t)gridDim.x * WG)
        if (!isfinite(a[i])) *flag = 1;
}

constexpr int NPART = 1024;

}  // namespace

// ====================================================================== launchers

void launch_elem_eig(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks, double* G,
                     int32_t* ranks, int32_t* status, double* scratch, int64_t scratch_stride, double rank_rtol,
                     double spsd_tol, int64_t n_max, hipStream_t st) {
    if (n_elem <= 0) return;
    // blocks up to NE_LDS: Jacobi with matrix and vectors in LDS; larger blocks: the
    // tridiagonal route (k_elem_eig_trd; 81 x 81 Q2 blocks: Jacobi took 0.67 s)
    const int64_t nl = std::min<int64_t>(n_max, NE_LDS);
    const int64_t lds = 2 * nl * nl * 8;
    hipLaunchKernelGGL(k_elem_eig, dim3((unsigned)n_elem), dim3(WG), (size_t)lds, st, elem_ptr, blk_off, blocks, G,
                       ranks, status, scratch, scratch_stride, rank_rtol, spsd_tol, lds);
    if (n_max > NE_LDS) {
        const size_t ld = (size_t)(2 * n_max + 64) * 8;
        const dim3 g((unsigned)n_elem);
        hipLaunchKernelGGL(k_elem_eig_trd<0>, g, dim3(WG), ld, st, elem_ptr, blk_off, blocks, G, ranks, status,
                           scratch, scratch_stride, rank_rtol, spsd_tol);
        hipLaunchKernelGGL(k_elem_eig_trd<1>, g, dim3(WG), ld, st, elem_ptr, blk_off, blocks, G, ranks, status,
                           scratch, scratch_stride, rank_rtol, spsd_tol);
        hipLaunchKernelGGL(k_elem_eig_trd<2>, g, dim3(WG), ld, st, elem_ptr, blk_off, blocks, G, ranks, status,
                           scratch, scratch_stride, rank_rtol, spsd_tol);
        hipLaunchKernelGGL(k_elem_eig_trd<3>, g, dim3(WG), ld, st, elem_ptr, blk_off, blocks, G, ranks, status,
                           scratch, scratch_stride, rank_rtol, spsd_tol);
    }
}

int64_t elem_eig_scratch_stride(int64_t n_max) {
    const int64_t jac = 3 * n_max * n_max;
    const int64_t trd = n_max > NE_LDS ? 2 * n_max * n_max + 4 * n_max + (int64_t)INVIT_SLOTS * n_max + 4096 : 0;
    return std::max(jac, trd);
}

void launch_elem_pchol(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                       double* G, int32_t* ranks, int32_t* status, double* scratch, int64_t scratch_stride,
                       double rank_rtol, double spsd_tol, hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_elem_pchol, dim3((unsigned)n_elem), dim3(WG), 0, st, elem_ptr, blk_off, blocks, G, ranks,
                       status, scratch, scratch_stride, rank_rtol, spsd_tol);
}

void launch_assemble_rows(int64_t n, const int64_t* d2e_ptr, const int32_t* d2e_elem, const int32_t* d2e_loc,
                          const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* blk_off,
                          const double* blocks, const double* factor, const int64_t* rowptr, const int32_t* col,
                          double* val, hipStream_t st, bool wave_rows) {
    if (n <= 0) return;
    if (wave_rows)
        hipLaunchKernelGGL(k_assemble_rows_wave, dim3(grid_for(n * 64)), dim3(WG), 0, st, n, d2e_ptr, d2e_elem,
                           d2e_loc, elem_ptr, elem_dofs, blk_off, blocks, factor, rowptr, col, val);
    else
        hipLaunchKernelGGL(k_assemble_rows, dim3(grid_for(n)), dim3(WG), 0, st, n, d2e_ptr, d2e_elem, d2e_loc,
                           elem_ptr, elem_dofs, blk_off, blocks, factor, rowptr, col, val);
}

void launch_theta_factor(int64_t n, const double* theta, const double* theta0, double* factor, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_theta_factor, dim3(grid_for(n)), dim3(WG), 0, st, n, theta, theta0, factor);
}

void launch_scale_blocks(int64_t n_elem, const int64_t* blk_off, const double* scale, double* blocks,
                         hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_scale_blocks, dim3((unsigned)std::min<int64_t>(n_elem, 65535 * 16)), dim3(WG), 0, st, n_elem,
                       blk_off, scale, blocks);
}

void launch_gram_rows(int64_t n_elem, const int64_t* perm_off, const int64_t* blk_off, const double* L,
                      const int32_t* perm, const int32_t* rank, double* G, hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_gram_rows, dim3((unsigned)std::min<int64_t>(n_elem, 65535 * 16)), dim3(WG), 0, st, n_elem,
                       perm_off, blk_off, L, perm, rank, G);
}

void launch_gram_csr_rows(int64_t n_elem, const int64_t* elem_ptr, const int64_t* src_off, const int64_t* blk_off,
                          const double* val, double* G, double* blocks, hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_gram_csr_rows, dim3((unsigned)std::min<int64_t>(n_elem, 65535 * 16)), dim3(WG), 0, st, n_elem,
                       elem_ptr, src_off, blk_off, val, G, blocks);
}

template <typename T, typename V>
void launch_elem_apply(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* tri_off,
                       const V* tri, int n_max, const T* x, V* ybuf, int64_t n, const int64_t* d2e_ptr,
                       const int32_t* e2y, const T* r_minus, T* y, hipStream_t st) {
    if (n_elem > 0) {
        if (n_max <= 32)
            hipLaunchKernelGGL((k_elem_tri_apply<T, V, 32, 1>), dim3(grid_for(n_elem, WG / 32)), dim3(WG), 0, st,
                               n_elem, elem_ptr, elem_dofs, tri_off, tri, x, ybuf);
        else if (n_max <= 64)
            hipLaunchKernelGGL((k_elem_tri_apply<T, V, 64, 1>), dim3(grid_for(n_elem, WG / 64)), dim3(WG), 0, st,
                               n_elem, elem_ptr, elem_dofs, tri_off, tri, x, ybuf);
        else
            hipLaunchKernelGGL((k_elem_tri_apply<T, V, 64, 2>), dim3(grid_for(n_elem, WG / 64)), dim3(WG), 0, st,
                               n_elem, elem_ptr, elem_dofs, tri_off, tri, x, ybuf);
    }
    if (n > 0)
        hipLaunchKernelGGL((k_elem_gather<T, V>), dim3(grid_for(n)), dim3(WG), 0, st, n, d2e_ptr, e2y, ybuf, r_minus,
                           y);
}
template void launch_elem_apply<double, double>(int64_t, const int64_t*, const int32_t*, const int64_t*,
                                                const double*, int, const double*, double*, int64_t, const int64_t*,
                                                const int32_t*, const double*, double*, hipStream_t);
template void launch_elem_apply<float, float>(int64_t, const int64_t*, const int32_t*, const int64_t*, const float*,
                                              int, const float*, float*, int64_t, const int64_t*, const int32_t*,
                                              const float*, float*, hipStream_t);
template void launch_elem_apply<float, double>(int64_t, const int64_t*, const int32_t*, const int64_t*,
                                               const double*, int, const float*, double*, int64_t, const int64_t*,
                                               const int32_t*, const float*, float*, hipStream_t);

void launch_pack_elem_tri(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                          const double* factor, const int64_t* tri_off, double* tri, float* tri32, hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_pack_elem_tri, dim3((unsigned)std::min<int64_t>(n_elem, 65535 * 16)), dim3(WG), 0, st,
                       n_elem, elem_ptr, blk_off, blocks, factor, tri_off, tri, tri32);
}

void launch_elem_bilinear(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* blk_off,
                          const double* blocks, const double* u, const double* v, int32_t nrhs, int64_t ld,
                          double scale, double* out, hipStream_t st) {
    if (n_elem <= 0) return;
    hipLaunchKernelGGL(k_elem_bilinear, dim3(grid_for(n_elem * 64)), dim3(WG), 0, st, n_elem, elem_ptr, elem_dofs,
                       blk_off, blocks, u, v, nrhs, ld, scale, out);
}

// blk_off[e] = sum_{f < e} n_f^2 for n_f = elem_ptr[f + 1] - elem_ptr[f], e = 0 .. n_elem:
// one workgroup, each thread sums a contiguous chunk, the chunk totals are scanned
// in LDS, then every thread writes its chunk's prefix sums.
__global__ void __launch_bounds__(1024) k_block_offsets(int64_t n_elem, const int64_t* elem_ptr, int64_t* blk_off) {
    __shared__ int64_t s[1024];
    const int t = (int)threadIdx.x;
    const int64_t chunk = (n_elem + 1023) / 1024;
    const int64_t a = min(n_elem, (int64_t)t * chunk), b = min(n_elem, a + chunk);
    int64_t sum = 0;
    for (int64_t e = a; e < b; ++e) {
        const int64_t m = elem_ptr[e + 1] - elem_ptr[e];
        sum += m * m;
    }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int64_t run = s[t] - sum;             // exclusive prefix of this chunk
    for (int64_t e = a; e < b; ++e) {
        blk_off[e] = run;
        const int64_t m = elem_ptr[e + 1] - elem_ptr[e];
        run += m * m;
    }
    if (t == 1023) blk_off[n_elem] = s[1023];
}

void launch_block_offsets(int64_t n_elem, const int64_t* elem_ptr, int64_t* blk_off, hipStream_t st) {
    hipLaunchKernelGGL(k_block_offsets, dim3(1), dim3(1024), 0, st, n_elem, elem_ptr, blk_off);
}

void launch_local_assemble(int32_t nbatch, const LocalArgs& a, int32_t max_m, hipStream_t st) {
    if (nbatch <= 0 || max_m <= 0) return;
    hipLaunchKernelGGL(k_local_assemble, dim3((max_m + ASM_CW - 1) / ASM_CW, nbatch), dim3(WG), 0, st, a);
}

void launch_local_eig(int32_t nbatch, const LocalArgs& a, int32_t max_nw, int first_phase, int last_phase,
                      hipStream_t st) {
    if (nbatch <= 0) return;
    // dynamic LDS: tridiagonal work vectors, cluster starts and dots, 2 |omega| doubles
    const size_t lds = (size_t)std::max(2 * max_nw, 4096) * sizeof(double);
    if (first_phase <= 0 && last_phase >= 0) hipLaunchKernelGGL(k_local_eig<0>, dim3(nbatch), dim3(WG), lds, st, a);
    if (first_phase <= 1 && last_phase >= 1) hipLaunchKernelGGL(k_local_eig<1>, dim3(nbatch), dim3(WG), lds, st, a);
    if (first_phase <= 2 && last_phase >= 2) hipLaunchKernelGGL(k_local_eig<2>, dim3(nbatch), dim3(WG), lds, st, a);
    if (first_phase <= 3 && last_phase >= 3) hipLaunchKernelGGL(k_local_eig<3>, dim3(nbatch), dim3(WG), lds, st, a);
}

void launch_stage_z(int32_t nbatch, const LocalArgs& a, hipStream_t st) {
    if (nbatch <= 0) return;
    hipLaunchKernelGGL(k_stage_z, dim3(nbatch), dim3(WG), 0, st, a);
}

void launch_views_max_diag(int32_t nv, const double* base, const View* v, double* out, hipStream_t st) {
    if (nv > 0) hipLaunchKernelGGL(k_views_max_diag, dim3(nv), dim3(WG), 0, st, base, v, out);
}
void launch_views_add_diag(int32_t nv, double* base, const View* v, const double* delta, hipStream_t st) {
    if (nv > 0) hipLaunchKernelGGL(k_views_add_diag, dim3(nv), dim3(WG), 0, st, base, v, delta);
}
void launch_views_symmetrize(int32_t nv, double* base, const View* v, hipStream_t st) {
    if (nv > 0) hipLaunchKernelGGL(k_views_symmetrize, dim3(64, nv), dim3(WG), 0, st, base, v);
}
void launch_views_identity(int32_t nv, double* base, const View* v, hipStream_t st) {
    if (nv > 0) hipLaunchKernelGGL(k_views_identity, dim3(256, nv), dim3(WG), 0, st, base, v);
}

void launch_z_compact(int32_t n_agg, const int64_t* agg_ptr, const int32_t* k, const int64_t* zst_off, const double* zst,
                      const int64_t* zoff, double* Z, double* Zc, float* Zc32, hipStream_t st) {
    if (n_agg <= 0) return;
    hipLaunchKernelGGL(k_z_compact, dim3(n_agg), dim3(WG), 0, st, agg_ptr, k, zst_off, zst, zoff, Z, Zc, Zc32);
}

void launch_build_pst(const PstArgs& g, hipStream_t st) {
    if (g.n_groups <= 0) return;
    hipLaunchKernelGGL(k_build_pst, dim3(g.n_groups), dim3(WG), 0, st, g);
}

void launch_dense_from_csr(int64_t off, int64_t n, const int64_t* rowptr, const int32_t* col, const double* val, double* D,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_dense_from_csr, dim3((unsigned)n), dim3(WG), 0, st, off, n, rowptr, col, val, D);
}

void launch_to_f32(int64_t n, const double* a, float* b, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(WG), 0, st, n, a, b);
}
void launch_to_f64(int64_t n, const float* a, double* b, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f64, dim3(grid_for(n)), dim3(WG), 0, st, n, a, b);
}

template <typename T, typename V>
void launch_csr_resid_rows(int64_t nrows, const int32_t* rows, const int64_t* rowptr, const int32_t* col, const V* val,
                           const T* x, const T* r, T* out, bool x_zero, int lanes, hipStream_t st,
                           const int64_t* scoff) {
    if (nrows <= 0) return;
    const int xz = x_zero ? 1 : 0;
    if (lanes >= 64)
        hipLaunchKernelGGL((k_csr_resid_rows<T, V, 64>), dim3(grid_for(nrows * 64)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, xz, scoff);
    else if (lanes >= 32)
        hipLaunchKernelGGL((k_csr_resid_rows<T, V, 32>), dim3(grid_for(nrows * 32)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, xz, scoff);
    else if (lanes >= 16)
        hipLaunchKernelGGL((k_csr_resid_rows<T, V, 16>), dim3(grid_for(nrows * 16)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, xz, scoff);
    else
        hipLaunchKernelGGL((k_csr_resid_rows<T, V, 8>), dim3(grid_for(nrows * 8)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, xz, scoff);
}
template <typename T, typename V>
void launch_sup_resid_blocks(int64_t nblk, const int32_t* blk, const int32_t* rows, const int64_t* rowptr,
                             const int32_t* scol, const int64_t* scoff, const V* val, const T* x, const T* r, T* out,
                             bool x_zero, int waves, hipStream_t st) {
    if (nblk <= 0) return;
    const int xz = x_zero ? 1 : 0;
    if (waves >= 4)
        hipLaunchKernelGGL((k_sup_resid_blocks<T, V, 4>), dim3(grid_for(nblk * 256)), dim3(WG), 0, st, nblk, blk,
                           rows, rowptr, scol, scoff, val, x, r, out, xz);
    else if (waves >= 2)
        hipLaunchKernelGGL((k_sup_resid_blocks<T, V, 2>), dim3(grid_for(nblk * 128)), dim3(WG), 0, st, nblk, blk,
                           rows, rowptr, scol, scoff, val, x, r, out, xz);
    else
        hipLaunchKernelGGL((k_sup_resid_blocks<T, V, 1>), dim3(grid_for(nblk * 64)), dim3(WG), 0, st, nblk, blk,
                           rows, rowptr, scol, scoff, val, x, r, out, xz);
}
template <typename T, typename V>
void launch_csr_spmv(int64_t n, const int64_t* rowptr, const int32_t* col, const V* val, const T* x, T* y,
                     const T* r_minus, int lanes, hipStream_t st, const int64_t* scoff) {
    if (n <= 0) return;
    if (lanes >= 64)
        hipLaunchKernelGGL((k_csr_spmv<T, V, 64>), dim3(grid_for(n * 64)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else if (lanes >= 32)
        hipLaunchKernelGGL((k_csr_spmv<T, V, 32>), dim3(grid_for(n * 32)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else if (lanes >= 16)
        hipLaunchKernelGGL((k_csr_spmv<T, V, 16>), dim3(grid_for(n * 16)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else
        hipLaunchKernelGGL((k_csr_spmv<T, V, 8>), dim3(grid_for(n * 8)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
}
template <typename T>
void launch_sub_symv(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                     const T* tiles, const T* rloc, const int64_t* scr_off, T* scr, int chl, hipStream_t st) {
    if (n_items <= 0) return;
    hipEvent_t e0, e1;
    if (take_launch_events(&e0, &e1))
        hipExtLaunchKernelGGL(k_sub_symv<T>, dim3((unsigned)n_items), dim3(WG), 0, st, e0, e1, 0, items, sub_off,
                              tp_off, tiles, rloc, scr_off, scr, chl);
    else
        hipLaunchKernelGGL(k_sub_symv<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, sub_off, tp_off, tiles,
                           rloc, scr_off, scr, chl);
}
template <typename T>
void launch_sub_finalize(int64_t r0, int64_t r1, const int32_t* pos_sub, const int64_t* sub_off,
                         const int64_t* scr_off, const T* scr, const int32_t* sub_dofs, T* x, bool accumulate,
                         int chl, int fl, hipStream_t st) {
    if (r1 <= r0) return;
    const int acc = accumulate ? 1 : 0;
    if (fl >= 32)
        hipLaunchKernelGGL((k_sub_finalize<T, 32>), dim3(grid_for(r1 - r0, WG / 32)), dim3(WG), 0, st, r0, r1,
                           pos_sub, sub_off, scr_off, scr, sub_dofs, x, acc, chl);
    else
        hipLaunchKernelGGL((k_sub_finalize<T, 8>), dim3(grid_for(r1 - r0, WG / 8)), dim3(WG), 0, st, r0, r1,
                           pos_sub, sub_off, scr_off, scr, sub_dofs, x, acc, chl);
}

template <typename T>
void launch_sub_finalize_tab(int64_t r0, int64_t r1, const int32_t* tab, const T* scr, const int32_t* sub_dofs, T* x,
                             int fl, hipStream_t st) {
    if (r1 <= r0) return;
    const int4* tb = reinterpret_cast<const int4*>(tab);
    if (fl >= 32)
        hipLaunchKernelGGL((k_sub_finalize_tab<T, 32>), dim3(grid_for(r1 - r0, WG / 32)), dim3(WG), 0, st, r0, r1, tb,
                           scr, sub_dofs, x);
    else
        hipLaunchKernelGGL((k_sub_finalize_tab<T, 8>), dim3(grid_for(r1 - r0, WG / 8)), dim3(WG), 0, st, r0, r1, tb,
                           scr, sub_dofs, x);
}
template void launch_sub_finalize_tab<double>(int64_t, int64_t, const int32_t*, const double*, const int32_t*, double*,
                                              int, hipStream_t);
template void launch_sub_finalize_tab<float>(int64_t, int64_t, const int32_t*, const float*, const int32_t*, float*,
                                             int, hipStream_t);

void launch_sub_fact(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                     const float* tiles, const float* rloc, const int64_t* scr_off, float* scr, int chl, int stash,
                     hipStream_t st) {
    if (n_items <= 0) return;
    stash = std::max(0, std::min(stash, SUB_FACT_MAX_STASH));
    static bool attr = false;
    if (!attr) {
        // allow the largest stash (the static LDS of the kernel comes on top)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sub_fact),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, SUB_FACT_MAX_STASH * 4096 * 4);
        attr = true;
    }
    hipLaunchKernelGGL(k_sub_fact, dim3((unsigned)n_items), dim3(WG), (size_t)stash * 4096 * 4, st, items, sub_off,
                       tp_off, tiles, rloc, scr_off, scr, chl, stash);
}

int64_t sub_symv_scratch_len(int64_t m, int chl) { return symv_scratch_len((int)((m + 63) / 64), chl); }

void sub_symv_items(int32_t s, int64_t m, int chl, std::vector<int32_t>& items) {
    const int nt = (int)((m + 63) / 64);
    for (int I = 0; I < nt; ++I)
        for (int ch = 0; ch * chl <= I; ++ch) {
            items.push_back(s);
            items.push_back(I);
            items.push_back(ch);
        }
}

void launch_pack_small(int32_t n_agg, const int64_t* sub_ptr, const int64_t* inv_off, const double* inv,
                       const int64_t* pk_off, double* pk, float* pk32, hipStream_t st) {
    if (n_agg <= 0) return;
    hipLaunchKernelGGL(k_pack_small, dim3((unsigned)n_agg), dim3(WG), 0, st, sub_ptr, inv_off, inv, pk_off, pk, pk32);
}

void launch_pack_tiles(int32_t n_agg, const int64_t* sub_ptr, const int64_t* inv_off, const double* inv,
                       const int64_t* tp_off, double* tiles, float* tiles32, hipStream_t st) {
    if (n_agg <= 0) return;
    hipLaunchKernelGGL(k_pack_tiles, dim3(n_agg == 1 ? 4096 : 64, n_agg), dim3(WG), 0, st, sub_ptr, inv_off, inv, tp_off,
                       tiles, tiles32);
}

template <typename T>
void launch_restrict(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                     const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* t, T* rc,
                     hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_restrict<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, agg_ptr, agg_dofs, zoff, k, coff,
                       Zc, t, rc);
}
template <typename T>
void launch_prolong(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                    const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                    hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_prolong<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, agg_ptr, agg_dofs, zoff, k, coff,
                       Zc, ec, x);
}
template <typename T>
void launch_zero(int64_t n, T* x, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(n)), dim3(WG), 0, st, n, x);
}

void launch_dot(int64_t n, const double* a, const double* b, double* partials, double* out, hipStream_t st) {
    unsigned nb = grid_for(n);
    if (nb > NPART) nb = NPART;
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(WG), 0, st, n, a, b, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, st, (int)nb, partials, out);
}

void launch_update_xr(int64_t n, const double* s_num, const double* s_den, const double* p, const double* q, double* x,
                      double* r, double* partials, double* out_rr, hipStream_t st) {
    unsigned nb = grid_for(n);
    if (nb > NPART) nb = NPART;
    hipLaunchKernelGGL(k_update_xr, dim3(nb), dim3(WG), 0, st, n, s_num, s_den, p, q, x, r, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, st, (int)nb, partials, out_rr);
}

void launch_update_p(int64_t n, const double* s_num, const double* s_den, const double* z, double* p, hipStream_t st) {
    hipLaunchKernelGGL(k_update_p, dim3(grid_for(n)), dim3(WG), 0, st, n, s_num, s_den, z, p);
}

void launch_copy(int64_t n, const double* a, double* b, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(WG), 0, st, n, a, b);
}

void launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(WG), 0, st, n, a, x, y);
}

void launch_check_finite(int64_t n, const double* a, int32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n)), dim3(WG), 0, st, n, a, flag);
}

#define LSDD_INST(T)                                                                                                  \
    template void launch_csr_resid_rows<T, T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const T*,     \
                                              const T*, const T*, T*, bool, int, hipStream_t, const int64_t*);        \
    template void launch_sup_resid_blocks<T, T>(int64_t, const int32_t*, const int32_t*, const int64_t*,              \
                                                const int32_t*, const int64_t*, const T*, const T*, const T*, T*,    \
                                                bool, int, hipStream_t);                                              \
    template void launch_csr_spmv<T, T>(int64_t, const int64_t*, const int32_t*, const T*, const T*, T*, const T*,    \
                                        int, hipStream_t, const int64_t*);                                            \
    template void launch_sub_symv<T>(int64_t, const int32_t*, const int64_t*, const int64_t*, const T*, const T*,    \
                                     const int64_t*, T*, int, hipStream_t);                                           \
    template void launch_sub_finalize<T>(int64_t, int64_t, const int32_t*, const int64_t*, const int64_t*, const T*, \
                                         const int32_t*, T*, bool, int, int, hipStream_t);                            \
    template void launch_restrict<T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const int64_t*,        \
                                     const int32_t*, const int64_t*, const T*, const T*, T*, hipStream_t);            \
    template void launch_prolong<T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const int64_t*,         \
                                    const int32_t*, const int64_t*, const T*, const T*, T*, hipStream_t);             \
    template void launch_zero<T>(int64_t, T*, hipStream_t);
LSDD_INST(double)
LSDD_INST(float)
template void launch_csr_resid_rows<float, double>(int64_t, const int32_t*, const int64_t*, const int32_t*,
                                                   const double*, const float*, const float*, float*, bool, int,
                                                   hipStream_t, const int64_t*);
template void launch_sup_resid_blocks<float, double>(int64_t, const int32_t*, const int32_t*, const int64_t*,
                                                     const int32_t*, const int64_t*, const double*, const float*,
                                                     const float*, float*, bool, int, hipStream_t);
template void launch_csr_spmv<float, double>(int64_t, const int64_t*, const int32_t*, const double*, const float*,
                                             float*, const float*, int, hipStream_t, const int64_t*);

}  // namespace lsdd
