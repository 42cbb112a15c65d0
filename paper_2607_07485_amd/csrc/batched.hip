// Batched tiled FP64 dense kernels (see batched.hpp).  Grid layout of every
// launch: blockIdx.y = view index, blockIdx.x = tile job inside that view;
// jobs past a view's own job count exit at once (views have different sizes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <stdexcept>
#include <string>

#include "batched.hpp"

namespace lsdd {

namespace {

constexpr int TB = 32;
constexpr int NT = 256;

__device__ inline int t_id() { return (int)threadIdx.x; }

__device__ inline void ld_tile(double (*t)[TB + 1], const double* a, const View& v, int r0, int c0) {
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = r0 + i, c = c0 + j;
        t[i][j] = (r < v.rows && c < v.cols) ? a[v.off + r + (int64_t)c * v.ld] : 0.0;
    }
}

__device__ inline void st_tile(const double (*t)[TB + 1], double* a, const View& v, int r0, int c0) {
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = r0 + i, c = c0 + j;
        if (r < v.rows && c < v.cols) a[v.off + r + (int64_t)c * v.ld] = t[i][j];
    }
}

__device__ inline int ntiles(int n) { return (n + TB - 1) / TB; }

// ---------------------------------------------------------------- Cholesky

__global__ void __launch_bounds__(NT) k_potrf_diag(double* base, const View* views, int kb, double* minpiv) {
    __shared__ double t[TB][TB + 1];
    __shared__ double s_min;
    const View v = views[blockIdx.y];
    const int n = v.rows;
    if (kb * TB >= n) return;
    const int r0 = kb * TB, nb = min(TB, n - r0);
    ld_tile(t, base, v, r0, r0);
    if (t_id() == 0) s_min = (kb == 0) ? INFINITY : minpiv[blockIdx.y];
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (t_id() == 0) {
            double d = t[j][j];
            s_min = fmin(s_min, (d == d) ? d : -1.0);
            t[j][j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double s = t[j][j];
        for (int i = j + 1 + t_id(); i < nb; i += NT) t[i][j] /= s;
        __syncthreads();
        for (int idx = t_id(); idx < nb * nb; idx += NT) {
            int i = idx % nb, k = idx / nb;
            if (i > j && k > j && i >= k) t[i][k] -= t[i][j] * t[k][j];
        }
        __syncthreads();
    }
    for (int idx = t_id(); idx < nb * nb; idx += NT) {
        int i = idx % nb, j = idx / nb;
        if (i >= j) base[v.off + (r0 + i) + (int64_t)(r0 + j) * v.ld] = t[i][j];
    }
    if (t_id() == 0) minpiv[blockIdx.y] = s_min;
}

// L_ib,kb = A_ib,kb L_kk^{-T}, ib = kb + 1 + blockIdx.x
__global__ void __launch_bounds__(NT) k_potrf_panel(double* base, const View* views, int kb) {
    __shared__ double L[TB][TB + 1];
    __shared__ double X[TB][TB + 1];
    const View v = views[blockIdx.y];
    const int nt = ntiles(v.rows);
    const int ib = kb + 1 + (int)blockIdx.x;
    if (ib >= nt) return;
    const int nb = min(TB, v.rows - kb * TB);
    ld_tile(L, base, v, kb * TB, kb * TB);
    ld_tile(X, base, v, ib * TB, kb * TB);
    __syncthreads();
    // x L^T = a per row: 8 threads per row split nothing; rows independent
    if (t_id() < TB) {
        const int r = t_id();
        for (int j = 0; j < nb; ++j) {
            double s = X[r][j];
            for (int k = 0; k < j; ++k) s -= X[r][k] * L[j][k];
            X[r][j] = s / L[j][j];
        }
    }
    __syncthreads();
    st_tile(X, base, v, ib * TB, kb * TB);
}

// A_ib,jb -= L_ib,kb L_jb,kb^T for kb < jb <= ib (lower tiles)
__global__ void __launch_bounds__(NT) k_potrf_update(double* base, const View* views, int kb) {
    __shared__ double Li[TB][TB + 1];
    __shared__ double Lj[TB][TB + 1];
    const View v = views[blockIdx.y];
    const int nt = ntiles(v.rows);
    const int m = nt - kb - 1;
    int t = (int)blockIdx.x;
    if (m <= 0 || t >= m * (m + 1) / 2) return;
    int jj = 0;
    while (t >= m - jj) { t -= m - jj; ++jj; }
    const int jb = kb + 1 + jj, ib = jb + t;
    ld_tile(Li, base, v, ib * TB, kb * TB);
    ld_tile(Lj, base, v, jb * TB, kb * TB);
    __syncthreads();
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = ib * TB + i, c = jb * TB + j;
        if (r < v.rows && c < v.cols && r >= c) {
            double s = 0.0;
#pragma unroll 8
            for (int k = 0; k < TB; ++k) s += Li[i][k] * Lj[j][k];
            base[v.off + r + (int64_t)c * v.ld] -= s;
        }
    }
}

// ---------------------------------------------------------------- triangular solves

// step s of L X = B (forward, kb = s) or L^T X = B (backward, kb = nt-1-s):
// solve the diagonal tile for every column tile of B.
__global__ void __launch_bounds__(NT) k_trsm_diag(const double* lbase, const View* lv, double* bbase, const View* bv,
                                                  int s, int trans) {
    __shared__ double L[TB][TB + 1];
    __shared__ double B[TB][TB + 1];
    const View l = lv[blockIdx.y], b = bv[blockIdx.y];
    const int nt = ntiles(l.rows);
    if (s >= nt) return;
    const int kb = trans ? nt - 1 - s : s;
    const int jc = (int)blockIdx.x;
    if (jc * TB >= b.cols) return;
    const int nb = min(TB, l.rows - kb * TB);
    ld_tile(L, lbase, l, kb * TB, kb * TB);
    ld_tile(B, bbase, b, kb * TB, jc * TB);
    __syncthreads();
    if (t_id() < TB) {
        const int c = t_id();
        if (!trans) {
            for (int i = 0; i < nb; ++i) {
                double v = B[i][c];
                for (int k = 0; k < i; ++k) v -= L[i][k] * B[k][c];
                B[i][c] = v / L[i][i];
            }
        } else {
            for (int i = nb - 1; i >= 0; --i) {
                double v = B[i][c];
                for (int k = i + 1; k < nb; ++k) v -= L[k][i] * B[k][c];
                B[i][c] = v / L[i][i];
            }
        }
    }
    __syncthreads();
    st_tile(B, bbase, b, kb * TB, jc * TB);
}

// update: forward B_ib -= L_ib,kb X_kb (ib > kb); backward B_ib -= L_kb,ib^T X_kb (ib < kb)
__global__ void __launch_bounds__(NT) k_trsm_update(const double* lbase, const View* lv, double* bbase, const View* bv,
                                                    int s, int trans) {
    __shared__ double L[TB][TB + 1];
    __shared__ double X[TB][TB + 1];
    const View l = lv[blockIdx.y], b = bv[blockIdx.y];
    const int nt = ntiles(l.rows);
    if (s >= nt) return;
    const int kb = trans ? nt - 1 - s : s;
    const int nct = ntiles(b.cols);
    const int nrow = trans ? kb : nt - kb - 1;     // tiles to update
    const int job = (int)blockIdx.x;
    if (job >= nrow * nct) return;
    const int ib = trans ? job % nrow : kb + 1 + job % nrow;
    const int jc = job / nrow;
    if (!trans) ld_tile(L, lbase, l, ib * TB, kb * TB);
    else ld_tile(L, lbase, l, kb * TB, ib * TB);
    ld_tile(X, bbase, b, kb * TB, jc * TB);
    __syncthreads();
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = ib * TB + i, c = jc * TB + j;
        if (r < b.rows && c < b.cols) {
            double acc = 0.0;
            if (!trans) {
#pragma unroll 8
                for (int k = 0; k < TB; ++k) acc += L[i][k] * X[k][j];
            } else {
#pragma unroll 8
                for (int k = 0; k < TB; ++k) acc += L[k][i] * X[k][j];
            }
            bbase[b.off + r + (int64_t)c * b.ld] -= acc;
        }
    }
}

// ---------------------------------------------------------------- C = beta C_in - alpha A^T B

__global__ void __launch_bounds__(NT) k_gemm_tn(const double* abase, const View* av, const double* bbase,
                                                const View* bv, const double* cinbase, const View* civ, double beta,
                                                double* coutbase, const View* cov, double alpha, int tri_k) {
    __shared__ double As[TB][TB + 1];
    __shared__ double Bs[TB][TB + 1];
    const View a = av[blockIdx.y], b = bv[blockIdx.y], co = cov[blockIdx.y];
    const int mt = ntiles(co.rows), ntt = ntiles(co.cols);
    const int job = (int)blockIdx.x;
    if (job >= mt * ntt) return;
    const int it = job % mt, jt = job / mt;
    const int kt = ntiles(a.rows);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int kb = tri_k ? max(it, jt) : 0; kb < kt; ++kb) {
        ld_tile(As, abase, a, kb * TB, it * TB);
        ld_tile(Bs, bbase, b, kb * TB, jt * TB);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int idx = t_id() + q * NT;
            int i = idx % TB, j = idx / TB;
            double s = 0.0;
#pragma unroll 8
            for (int k = 0; k < TB; ++k) s += As[k][i] * Bs[k][j];
            acc[q] += s;
        }
        __syncthreads();
    }
    for (int q = 0; q < 4; ++q) {
        int idx = t_id() + q * NT;
        int i = idx % TB, j = idx / TB;
        int r = it * TB + i, c = jt * TB + j;
        if (r < co.rows && c < co.cols) {
            double v = -alpha * acc[q];
            if (beta != 0.0) {
                const View ci = civ[blockIdx.y];
                v += beta * cinbase[ci.off + r + (int64_t)c * ci.ld];
            }
            coutbase[co.off + r + (int64_t)c * co.ld] = v;
        }
    }
}

// ---------------------------------------------------------------- transpose

__global__ void __launch_bounds__(NT) k_transpose(double* base, const View* views) {
    __shared__ double P[TB][TB + 1];
    __shared__ double Q[TB][TB + 1];
    const View v = views[blockIdx.y];
    const int nt = ntiles(v.rows);
    int t = (int)blockIdx.x;
    if (t >= nt * (nt + 1) / 2) return;
    int jt = 0;
    while (t > jt) { t -= jt + 1; ++jt; }
    const int it = t;   // it <= jt
    ld_tile(P, base, v, it * TB, jt * TB);
    ld_tile(Q, base, v, jt * TB, it * TB);
    __syncthreads();
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = it * TB + i, c = jt * TB + j;
        if (r < v.rows && c < v.cols) base[v.off + r + (int64_t)c * v.ld] = Q[j][i];
        int r2 = jt * TB + i, c2 = it * TB + j;
        if (r2 < v.rows && c2 < v.cols) base[v.off + r2 + (int64_t)c2 * v.ld] = P[j][i];
    }
}

void chk(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

View* Batched::put(int slot, const std::vector<View>& v) {
    if (v.size() > 65535) throw std::runtime_error("batched: more than 65535 views in one launch");
    if (v.size() > slot_cap) {
        for (View*& p : d_slot)
            if (p) release(ctx, p);
        slot_cap = std::max<size_t>(v.size(), 64);
        for (View*& p : d_slot) p = (View*)alloc(ctx, slot_cap * sizeof(View));
    }
    chk(hipMemcpyAsync(d_slot[slot], v.data(), v.size() * sizeof(View), hipMemcpyHostToDevice, st), "view upload");
    chk(hipStreamSynchronize(st), "view upload sync");
    return d_slot[slot];
}

void Batched::free_all() {
    for (View*& p : d_slot) {
        if (p) release(ctx, p);
        p = nullptr;
    }
    slot_cap = 0;
}

static int max_tiles(const std::vector<View>& v, bool rows) {
    int m = 0;
    for (const View& x : v) m = std::max(m, ((rows ? x.rows : x.cols) + TB - 1) / TB);
    return m;
}

void Batched::potrf(double* base, const std::vector<View>& a, double* d_minpiv) {
    if (a.empty()) return;
    View* dv = put(0, a);
    const unsigned nm = (unsigned)a.size();
    const int nt = max_tiles(a, true);
    for (int kb = 0; kb < nt; ++kb) {
        hipLaunchKernelGGL(k_potrf_diag, dim3(1, nm), dim3(NT), 0, st, base, dv, kb, d_minpiv);
        const int below = nt - kb - 1;
        if (below > 0) {
            hipLaunchKernelGGL(k_potrf_panel, dim3(below, nm), dim3(NT), 0, st, base, dv, kb);
            hipLaunchKernelGGL(k_potrf_update, dim3(below * (below + 1) / 2, nm), dim3(NT), 0, st, base, dv, kb);
        }
    }
    chk(hipGetLastError(), "batched potrf");
}

void Batched::trsm(const double* lbase, const std::vector<View>& l, double* bbase, const std::vector<View>& b,
                   bool trans) {
    if (l.empty()) return;
    View* d1 = put(0, l);
    View* d2 = put(1, b);
    const unsigned nm = (unsigned)l.size();
    const int nt = max_tiles(l, true);
    const int nct = max_tiles(b, false);
    if (nct == 0) return;
    for (int s = 0; s < nt; ++s) {
        hipLaunchKernelGGL(k_trsm_diag, dim3(nct, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, s, trans ? 1 : 0);
        const int jobs = (nt - 1) * nct;
        if (jobs > 0)
            hipLaunchKernelGGL(k_trsm_update, dim3(jobs, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, s, trans ? 1 : 0);
    }
    chk(hipGetLastError(), "batched trsm");
}

void Batched::gemm_tn(const double* abase, const std::vector<View>& a, const double* bbase, const std::vector<View>& b,
                      const double* cinbase, const std::vector<View>& cin, double beta, double* coutbase,
                      const std::vector<View>& cout, double alpha, bool tri_k) {
    if (a.empty()) return;
    View* d1 = put(0, a);
    View* d2 = put(1, b);
    View* d3 = put(2, cout);
    View* d4 = beta != 0.0 ? put(3, cin) : d3;
    const unsigned nm = (unsigned)a.size();
    int mt = 0;
    for (const View& x : cout) mt = std::max(mt, ((x.rows + TB - 1) / TB) * ((x.cols + TB - 1) / TB));
    if (mt == 0) return;
    hipLaunchKernelGGL(k_gemm_tn, dim3(mt, nm), dim3(NT), 0, st, abase, d1, bbase, d2, cinbase, d4, beta, coutbase,
                       d3, alpha, tri_k ? 1 : 0);
    chk(hipGetLastError(), "batched gemm_tn");
}

void Batched::transpose(double* base, const std::vector<View>& a) {
    if (a.empty()) return;
    View* d1 = put(0, a);
    const unsigned nm = (unsigned)a.size();
    const int nt = max_tiles(a, true);
    hipLaunchKernelGGL(k_transpose, dim3(nt * (nt + 1) / 2, nm), dim3(NT), 0, st, base, d1);
    chk(hipGetLastError(), "batched transpose");
}

}  // namespace lsdd
