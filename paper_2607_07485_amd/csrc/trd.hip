// Blocked Householder tridiagonalisation of the larger local spectral problems
// (C = L^{-1} S~ L^{-T} of an aggregate), many matrices per launch and many
// workgroups per matrix.
//
// The reduction T = Q^T C Q is the one the single-workgroup path computes
// (reflector j from column j below the diagonal, tau_j, d, e), but the
// rank-2 updates of the trailing matrix are delayed over panels of TRD_NB
// columns: inside a panel, column j is corrected by the panel's earlier
// reflectors (V, W) and the matrix-vector product with the trailing block is
// corrected the same way; after the panel one symmetric rank-2k update
// C22 -= V W^T + W V^T runs on the FP64 matrix cores.  Per column:
//   k_trd_col   (one workgroup per matrix): finish the previous W column,
//               correct column j, form reflector v_j (stored in column j, with
//               an explicit 1 on the subdiagonal), dots W^T v and V^T v;
//   k_trd_symv  (many workgroups per matrix): w = tau (C22 v - V (W^T v)
//               - W (V^T v)), one wave per column of C22.
// Per panel: k_trd_fin (finish the last W column), k_trd_update.
//
// Storage per matrix: C (n x n, both triangles kept exactly symmetric), the
// tridiagonal d, e, tau in the T scratch, V and W (n x TRD_NB each,
// column-major, so row sweeps over one column are coalesced) and the dots in
// the v_buf slot (n^2 doubles, n > 2 TRD_NB).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <vector>

#include "dense.hpp"
#include "kernels.hpp"
#include "mgemm.hpp"

namespace lsdd {

namespace {

constexpr int WG = LSDD_WG;
constexpr int NB = TRD_NB;
constexpr int CPW = 4;               // columns per wave in k_trd_symv
constexpr int CPG = CPW * WG / 64;   // columns per workgroup

struct Mat {
    int n;
    double* a;
    double* d;
    double* e;
    double* tau;
    double* V;
    double* W;
    double* zw;
    double* zv;
};

__device__ inline Mat mat_of(const LocalArgs& A, int b) {
    Mat m;
    const int ag = A.first + b;
    m.n = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    m.a = A.s_buf + A.sq_off[b];
    double* T = A.t_buf + A.t_off[b];
    m.d = T;
    m.e = T + m.n;
    m.tau = T + 2 * m.n;
    m.V = A.v_buf + A.sq_off[b];
    m.W = m.V + (int64_t)NB * m.n;
    m.zw = m.W + (int64_t)NB * m.n;
    m.zv = m.zw + NB;
    return m;
}

// W(:, q) <- w - (tau_jp / 2) (w . v) v for the raw w of reflector jp
__device__ inline void finish_w(const Mat& m, int jp, int q, double* red) {
    double s = 0.0;
    const double* vq = m.V + (int64_t)q * m.n;
    double* wq = m.W + (int64_t)q * m.n;
    for (int i = jp + 1 + tid(); i < m.n; i += WG) s += wq[i] * vq[i];
    s = wg_sum(s, red);
    const double K = 0.5 * m.tau[jp] * s;
    for (int i = jp + 1 + tid(); i < m.n; i += WG) wq[i] -= K * vq[i];
    __syncthreads();
}

__global__ void __launch_bounds__(WG) k_trd_col(LocalArgs A, const int32_t* big, int j, int j0) {
    __shared__ double red[WG / 64];
    __shared__ double rowvw[2 * NB];
    __shared__ double part[WG / 64][2 * NB];
    const Mat m = mat_of(A, big[blockIdx.x]);
    const int n = m.n;
    if (j + 2 >= n) return;
    const int p = j - j0;
    if (p > 0) finish_w(m, j - 1, p - 1, red);
    // column j (rows j..n-1) with the panel's earlier reflectors applied
    if (tid() < p) {
        rowvw[tid()] = m.V[j + (int64_t)tid() * n];
        rowvw[NB + tid()] = m.W[j + (int64_t)tid() * n];
    }
    __syncthreads();
    double* col = m.a + (int64_t)j * n;
    for (int i = j + tid(); i < n; i += WG) {
        double s = col[i];
        for (int q = 0; q < p; ++q) s -= m.V[i + (int64_t)q * n] * rowvw[NB + q] + m.W[i + (int64_t)q * n] * rowvw[q];
        col[i] = s;
    }
    __syncthreads();
    // reflector from x = col[j+1 .. n-1]
    const int mm = n - j - 1;
    double* x = col + j + 1;
    double s2 = 0.0;
    for (int i = 1 + tid(); i < mm; i += WG) s2 += x[i] * x[i];
    s2 = wg_sum(s2, red);
    const double alpha = x[0];
    double t = 0.0, beta = alpha, sc = 0.0;
    if (s2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + s2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
    }
    if (tid() == 0) {
        m.d[j] = col[j];
        m.e[j] = beta;
        m.tau[j] = t;
    }
    __syncthreads();
    double* vp = m.V + (int64_t)p * n;
    for (int i = tid(); i < mm; i += WG) {
        const double vi = (i == 0) ? 1.0 : (s2 > 0.0 ? x[i] * sc : 0.0);
        x[i] = vi;
        vp[j + 1 + i] = vi;
    }
    for (int i = j0 + tid(); i <= j; i += WG) {
        vp[i] = 0.0;
        m.W[i + (int64_t)p * n] = 0.0;
    }
    __syncthreads();
    // zw_q = W(j+1:, q) . v, zv_q = V(j+1:, q) . v for q < p
    const int w = tid() >> 6, l = tid() & 63;
    for (int q0 = 0; q0 < p; q0 += 8) {
        double aw[8], av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) aw[u] = av[u] = 0.0;
        for (int i = j + 1 + tid(); i < n; i += WG) {
            const double vi = x[i - j - 1];
            // columns past p re-read column p - 1 (the loads stay unconditional and in
            // flight together) and are not added
            double ww[8], vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t qc = min(q0 + u, p - 1);
                ww[u] = m.W[i + qc * n];
                vv[u] = m.V[i + qc * n];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u < p) {
                    aw[u] += ww[u] * vi;
                    av[u] += vv[u] * vi;
                }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            aw[u] = wave_sum(aw[u]);
            av[u] = wave_sum(av[u]);
        }
        if (l == 0)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                part[w][q0 + u] = aw[u];
                part[w][NB + q0 + u] = av[u];
            }
    }
    __syncthreads();
    if (tid() < p) {
        double sw = 0.0, sv = 0.0;
        for (int r = 0; r < WG / 64; ++r) {
            sw += part[r][tid()];
            sv += part[r][NB + tid()];
        }
        m.zw[tid()] = sw;
        m.zv[tid()] = sv;
    }
}

__global__ void __launch_bounds__(WG) k_trd_symv(LocalArgs A, const int32_t* big, int j, int j0) {
    extern __shared__ double s_v[];    // v (n - j - 1), then zw, zv
    const Mat m = mat_of(A, big[blockIdx.y]);
    const int n = m.n;
    if (j + 2 >= n) return;
    const int mm = n - j - 1;
    const int c0 = (int)blockIdx.x * CPG;
    if (c0 >= mm) return;
    const int p = j - j0;
    const double* v = m.a + (int64_t)j * n + j + 1;
    double* zz = s_v + mm;
    for (int i = tid(); i < mm; i += WG) s_v[i] = v[i];
    if (tid() < p) {
        zz[tid()] = m.zw[tid()];
        zz[NB + tid()] = m.zv[tid()];
    }
    __syncthreads();
    const double t = m.tau[j];
    const int w = tid() >> 6, l = tid() & 63;
    for (int cc = 0; cc < CPW; ++cc) {
        const int c = c0 + w * CPW + cc;
        if (c >= mm) break;
        const double* cp = m.a + (int64_t)(j + 1 + c) * n + j + 1;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = l;
        for (; i + 192 < mm; i += 256) {
            s0 += cp[i] * s_v[i];
            s1 += cp[i + 64] * s_v[i + 64];
            s2 += cp[i + 128] * s_v[i + 128];
            s3 += cp[i + 192] * s_v[i + 192];
        }
        for (; i < mm; i += 64) s0 += cp[i] * s_v[i];
        // the panel's correction V (W^T v) + W (V^T v) of row gi, one term per lane
        // (p <= NB < 64), folded into the same wave reduction
        const int gi = j + 1 + c;
        double corr = 0.0;
        if (l < p) corr = m.V[gi + (int64_t)l * n] * zz[l] + m.W[gi + (int64_t)l * n] * zz[NB + l];
        const double s = wave_sum(((s0 + s1) + (s2 + s3)) - corr);
        if (l == 0) m.W[gi + (int64_t)p * n] = t * s;
    }
}

__global__ void __launch_bounds__(WG) k_trd_fin(LocalArgs A, const int32_t* big, int j0) {
    __shared__ double red[WG / 64];
    const Mat m = mat_of(A, big[blockIdx.x]);
    const int pc = min(NB, m.n - 2 - j0);
    if (pc <= 0) return;
    finish_w(m, j0 + pc - 1, pc - 1, red);
}

// C[r0:, r0:] -= V W^T + W V^T over lower tile pairs, stored to both triangles
__global__ void __launch_bounds__(WG) k_trd_update(LocalArgs A, const int32_t* big, int j0) {
    __shared__ mg::Smem sm;
    const Mat m = mat_of(A, big[blockIdx.y]);
    const int n = m.n;
    const int pc = min(NB, n - 2 - j0);
    if (pc <= 0) return;
    const int r0 = j0 + pc, M = n - r0;
    const int mt = (M + mg::T - 1) / mg::T;
    int job = (int)blockIdx.x;
    if (job >= mt * (mt + 1) / 2) return;
    int jt = 0;
    while (job >= mt - jt) {
        job -= mt - jt;
        ++jt;
    }
    const int it = jt + job;
    const double* Vr = m.V + r0;                 // (k = reflector, i = row) at Vr[i + k n]
    const double* Wr = m.W + r0;
    mg::d4 acc[2][2];
    mg::zero(acc);
    mg::tile_mma<mg::IMAJ, mg::IMAJ>(sm, Vr, n, it * mg::T, M, Wr, n, jt * mg::T, M, 0, pc, acc);
    mg::tile_mma<mg::IMAJ, mg::IMAJ>(sm, Wr, n, it * mg::T, M, Vr, n, jt * mg::T, M, 0, pc, acc);
    double old[2][2][4];   // loaded before use, addresses clamped (no conditional loads)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t rr = r0 + min(it * mg::T + mg::acc_row(p, e), M - 1);
                const int64_t cc = r0 + min(jt * mg::T + mg::acc_col(q), M - 1);
                old[p][q][e] = m.a[rr + cc * n];
            }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = it * mg::T + mg::acc_row(p, e), c = jt * mg::T + mg::acc_col(q);
                if (i < M && c < M && i >= c) {
                    const int64_t rr = r0 + i, cc = r0 + c;
                    const double x = old[p][q][e] - acc[p][q][e];
                    m.a[rr + cc * n] = x;
                    if (i != c) m.a[cc + rr * n] = x;
                }
            }
}

__global__ void k_trd_tail(LocalArgs A, const int32_t* big) {
    const Mat m = mat_of(A, big[blockIdx.x]);
    const int n = m.n;
    if (tid() == 0 && n >= 3) {
        m.d[n - 2] = m.a[(n - 2) + (int64_t)(n - 2) * n];
        m.e[n - 2] = m.a[(n - 1) + (int64_t)(n - 2) * n];
        m.d[n - 1] = m.a[(n - 1) + (int64_t)(n - 1) * n];
    }
}

// All eigenvalues of the large problems' tridiagonal matrices by bisection,
// WG of them per workgroup (before the mode-count phase of k_local_eig).
__global__ void __launch_bounds__(WG) k_trd_bisect(LocalArgs A, const int32_t* big) {
    __shared__ double red[WG / 64];
    const int b = big[blockIdx.y];
    const int ag = A.first + b;
    const int n = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    const int i0 = (int)blockIdx.x * WG;
    if (i0 >= n) return;
    const double* T = A.t_buf + A.t_off[b];
    wg_bisect_range(T, T + n, n, A.mu + A.mu_off[ag], i0, min(n, i0 + WG), red);
}

// Retained eigenvectors of the large problems' tridiagonal matrices by
// inverse iteration: workgroup x takes the eigenvalue indices [64x, 64x + 64)
// (singletons one per thread, and the clusters that start there).
__global__ void __launch_bounds__(WG) k_trd_invit(LocalArgs A, const int32_t* big, const int64_t* iw_off,
                                                  double* iw) {
    __shared__ double red[WG / 64];
    __shared__ int s_ncl;
    __shared__ mg::Smem sm;
    extern __shared__ double s_dyn[];
    const int b = big[blockIdx.y];
    const int ag = A.first + b;
    const int n = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    const int kk = A.k_out[ag];
    const int r0 = (int)blockIdx.x * 64;
    if (r0 >= kk) return;
    const double* T = A.t_buf + A.t_off[b];
    const double* d = T;
    const double* e = T + n;
    double tnorm = 0.0;
    for (int i = tid(); i < n; i += WG)
        tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
    tnorm = wg_max(tnorm, red);
    double* ws = iw + iw_off[blockIdx.y] + (int64_t)blockIdx.x * ((int64_t)INVIT_SLOTS * n + 4096);
    wg_inverse_iteration_range(d, e, n, A.mu + A.mu_off[ag], kk, r0, min(kk, r0 + 64), A.w1 + A.ws_off[b], ws,
                               ws + (int64_t)INVIT_SLOTS * n, fmax(tnorm, 1e-300), (int*)(s_dyn + 64), s_dyn, red,
                               &s_ncl, &sm);
}

// Retained eigenvectors x <- Q x (Q = H_0 ... H_{n-3}) for the large
// problems: one wave per vector (VS = W1, n x k, ld n), reflectors applied
// from the last to the first, four per round: with the dots d_k = v_k^T x and
// the cross products c_kl = v_k^T v_l of reflectors j, j-1, j-2, j-3 (k = 0..3)
// gathered in one pass, s_k = tau_k (d_k - sum_{l<k} s_l c_kl) are the
// multipliers of applying them one after the other, and x -= sum_k s_k v_k.
// Lane l owns the rows r = l (mod 64) of its vector, so no lane reads another
// lane's writes.
__global__ void __launch_bounds__(WG) k_trd_backtransform(LocalArgs A, const int32_t* big) {
    const int b = big[blockIdx.y];
    const int ag = A.first + b;
    const int n = (int)(A.agg_ptr[ag + 1] - A.agg_ptr[ag]);
    const int kk = A.k_out[ag];
    const int c = (int)blockIdx.x * (WG / 64) + (tid() >> 6);
    if (c >= kk) return;
    const int l = tid() & 63;
    const double* a = A.s_buf + A.sq_off[b];
    const double* tau = A.t_buf + A.t_off[b] + 2 * n;
    double* x = A.w1 + A.ws_off[b] + (int64_t)c * n;
    // entry r of reflector jj: 1 at jj + 1, stored below it, 0 above
    auto vr = [&](int jj, int r) { return r == jj + 1 ? 1.0 : (r > jj + 1 ? a[r + (int64_t)jj * n] : 0.0); };
    int j = n - 3;
    for (; j >= 3; j -= 4) {
        const int r0 = j - 2 + ((l - (j - 2)) % 64 + 64) % 64;     // first owned row >= j - 2
        double d[4] = {0.0, 0.0, 0.0, 0.0}, cc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int r = r0; r < n; r += 64) {
            const double xr = x[r];
            double v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = vr(j - k, r);
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] += v[k] * xr;
            cc[0] += v[1] * v[0];
            cc[1] += v[2] * v[0];
            cc[2] += v[2] * v[1];
            cc[3] += v[3] * v[0];
            cc[4] += v[3] * v[1];
            cc[5] += v[3] * v[2];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = wave_sum(d[k]);
#pragma unroll
        for (int q = 0; q < 6; ++q) cc[q] = wave_sum(cc[q]);
        double sk[4];
        sk[0] = tau[j] * d[0];
        sk[1] = tau[j - 1] * (d[1] - sk[0] * cc[0]);
        sk[2] = tau[j - 2] * (d[2] - sk[0] * cc[1] - sk[1] * cc[2]);
        sk[3] = tau[j - 3] * (d[3] - sk[0] * cc[3] - sk[1] * cc[4] - sk[2] * cc[5]);
        for (int r = r0; r < n; r += 64) {
            double y = x[r];
#pragma unroll
            for (int k = 0; k < 4; ++k) y -= sk[k] * vr(j - k, r);
            x[r] = y;
        }
    }
    for (; j >= 0; --j) {
        const double t = tau[j];
        if (t == 0.0) continue;
        const double* v = a + (int64_t)j * n;
        const int r0 = j + 1 + ((l - (j + 1)) % 64 + 64) % 64;     // first owned row > j
        double s = 0.0;
        for (int r = r0; r < n; r += 64) s += (r == j + 1 ? 1.0 : v[r]) * x[r];
        s = wave_sum(s) * t;
        for (int r = r0; r < n; r += 64) x[r] -= s * (r == j + 1 ? 1.0 : v[r]);
    }
}

}  // namespace

void launch_local_backtransform_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                        hipStream_t st) {
    const int nbig = (int)sizes.size();
    if (nbig == 0) return;
    int max_n = 0;
    for (int32_t s : sizes) max_n = std::max(max_n, (int)s);
    hipLaunchKernelGGL(k_trd_backtransform, dim3((max_n + WG / 64 - 1) / (WG / 64), nbig), dim3(WG), 0, st, a, d_big);
}

void launch_local_invit_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                const std::vector<int32_t>& ks, const int64_t* d_iw_off, double* iw, hipStream_t st) {
    const int nbig = (int)sizes.size();
    int max_n = 0, max_g = 0;
    for (int i = 0; i < nbig; ++i) {
        max_n = std::max(max_n, (int)sizes[i]);
        max_g = std::max(max_g, (ks[i] + 63) / 64);
    }
    if (max_g == 0) return;
    const size_t lds = 64 * sizeof(double) + (size_t)(max_n + 1) * sizeof(int);   // dots, cluster starts
    hipLaunchKernelGGL(k_trd_invit, dim3(max_g, nbig), dim3(WG), lds, st, a, d_big, d_iw_off, iw);
}

void launch_local_tridiag_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                  hipStream_t st) {
    const int nbig = (int)sizes.size();
    if (nbig == 0) return;
    int max_n = 0;
    for (int32_t s : sizes) {
        if (s <= 2 * NB + 1) throw std::runtime_error("blocked tridiagonalisation needs n > 2 * TRD_NB + 1");
        max_n = std::max(max_n, (int)s);
    }
    const size_t lds = (size_t)(max_n + 2 * NB) * sizeof(double);
    for (int j0 = 0; j0 < max_n - 2; j0 += NB) {
        const int j1 = std::min(j0 + NB, max_n - 2);
        for (int j = j0; j < j1; ++j) {
            hipLaunchKernelGGL(k_trd_col, dim3(nbig), dim3(WG), 0, st, a, d_big, j, j0);
            const int mm = max_n - j - 1;
            hipLaunchKernelGGL(k_trd_symv, dim3((mm + CPG - 1) / CPG, nbig), dim3(WG), lds, st, a, d_big, j, j0);
        }
        hipLaunchKernelGGL(k_trd_fin, dim3(nbig), dim3(WG), 0, st, a, d_big, j0);
        int64_t jobs = 0;
        for (int32_t n : sizes) {
            const int pc = std::min(NB, (int)n - 2 - j0);
            if (pc <= 0) continue;
            const int64_t mt = (n - j0 - pc + mg::T - 1) / mg::T;
            jobs = std::max(jobs, mt * (mt + 1) / 2);
        }
        if (jobs > 0) hipLaunchKernelGGL(k_trd_update, dim3((unsigned)jobs, nbig), dim3(WG), 0, st, a, d_big, j0);
    }
    hipLaunchKernelGGL(k_trd_tail, dim3(nbig), dim3(64), 0, st, a, d_big);
    hipLaunchKernelGGL(k_trd_bisect, dim3((max_n + WG - 1) / WG, nbig), dim3(WG), 0, st, a, d_big);
}

}  // namespace lsdd
