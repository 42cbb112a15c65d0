// Workgroup-cooperative dense linear algebra for the batched local problems.
//
// Every routine is executed by all threads of one workgroup (blockDim.x ==
// LSDD_WG) on one matrix; matrices are column-major with a leading dimension
// and may live in LDS or in global memory (flat addressing).  The routines
// synchronise internally and leave the workgroup synchronised on return.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#define LSDD_WG 256

namespace lsdd {

__device__ inline int tid() { return (int)threadIdx.x; }

// ---------------------------------------------------------------- reductions

template <typename T>
__device__ inline T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ inline T wave_max(T v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Workgroup sum; `red` is LDS scratch of at least LSDD_WG/64 entries.
template <typename T>
__device__ inline T wg_sum(T v, T* red) {
    v = wave_sum(v);
    const int w = tid() >> 6, l = tid() & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < LSDD_WG / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

template <typename T>
__device__ inline T wg_max(T v, T* red) {
    v = wave_max(v);
    const int w = tid() >> 6, l = tid() & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T s = red[0];
    for (int i = 1; i < LSDD_WG / 64; ++i) s = fmax(s, red[i]);
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- elementary ops

__device__ inline void wg_zero(double* a, long long count) {
    for (long long i = tid(); i < count; i += LSDD_WG) a[i] = 0.0;
    __syncthreads();
}

__device__ inline void wg_identity(double* a, int ld, int n) {
    for (long long idx = tid(); idx < (long long)n * n; idx += LSDD_WG) {
        int i = (int)(idx % n), j = (int)(idx / n);
        a[i + (long long)j * ld] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
}

// a <- (a + a^T)/2 on an n x n block.
__device__ inline void wg_symmetrize(double* a, int ld, int n) {
    for (long long idx = tid(); idx < (long long)n * n; idx += LSDD_WG) {
        int i = (int)(idx % n), j = (int)(idx / n);
        if (i < j) {
            double s = 0.5 * (a[i + (long long)j * ld] + a[j + (long long)i * ld]);
            a[i + (long long)j * ld] = s;
            a[j + (long long)i * ld] = s;
        }
    }
    __syncthreads();
}

// In-place transpose of a square n x n block.
__device__ inline void wg_transpose(double* a, int ld, int n) {
    for (long long idx = tid(); idx < (long long)n * n; idx += LSDD_WG) {
        int i = (int)(idx % n), j = (int)(idx / n);
        if (i < j) {
            double t = a[i + (long long)j * ld];
            a[i + (long long)j * ld] = a[j + (long long)i * ld];
            a[j + (long long)i * ld] = t;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- Cholesky

// Right-looking Cholesky A = L L^T of an SPD n x n matrix, lower triangle in
// place.  Returns the smallest pivot d_j = L_jj^2 seen (<= 0 or NaN: failed at
// that column, the factor is incomplete).  `sh` is LDS scratch of 2 doubles.
__device__ inline double wg_potrf(double* a, int ld, int n, double* sh) {
    if (tid() == 0) sh[1] = INFINITY;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid() == 0) {
            double d = a[j + (long long)j * ld];
            sh[1] = fmin(sh[1], d);
            if (!(d > 0.0)) sh[1] = (d == d) ? d : -1.0;
            double s = (d > 0.0) ? sqrt(d) : 0.0;
            a[j + (long long)j * ld] = s;
            sh[0] = s;
        }
        __syncthreads();
        const double s = sh[0];
        if (!(s > 0.0)) {
            double r = sh[1];
            __syncthreads();
            return r;
        }
        const double inv = 1.0 / s;
        double* cj = a + (long long)j * ld;
        for (int i = j + 1 + tid(); i < n; i += LSDD_WG) cj[i] *= inv;
        __syncthreads();
        const int m = n - j - 1;
        for (long long idx = tid(); idx < (long long)m * m; idx += LSDD_WG) {
            int ii = (int)(idx % m), kk = (int)(idx / m);
            if (ii >= kk) {
                int i = j + 1 + ii, k = j + 1 + kk;
                a[i + (long long)k * ld] -= cj[i] * cj[k];
            }
        }
        __syncthreads();
    }
    double r = sh[1];
    __syncthreads();
    return r;
}

// Forward solve L X = B in place (L lower n x n, B n x m).
__device__ inline void wg_trsm_lower(const double* L, int ldl, int n, double* B, int ldb, int m) {
    for (int j = 0; j < n; ++j) {
        const double inv = 1.0 / L[j + (long long)j * ldl];
        for (int c = tid(); c < m; c += LSDD_WG) B[j + (long long)c * ldb] *= inv;
        __syncthreads();
        const int r = n - j - 1;
        if (r > 0) {
            const double* lj = L + (long long)j * ldl;
            for (long long idx = tid(); idx < (long long)r * m; idx += LSDD_WG) {
                int ii = (int)(idx % r), c = (int)(idx / r);
                int i = j + 1 + ii;
                B[i + (long long)c * ldb] -= lj[i] * B[j + (long long)c * ldb];
            }
        }
        __syncthreads();
    }
}

// Backward solve L^T X = B in place (L lower n x n, B n x m).
__device__ inline void wg_trsm_lower_t(const double* L, int ldl, int n, double* B, int ldb, int m) {
    for (int j = n - 1; j >= 0; --j) {
        const double inv = 1.0 / L[j + (long long)j * ldl];
        for (int c = tid(); c < m; c += LSDD_WG) B[j + (long long)c * ldb] *= inv;
        __syncthreads();
        if (j > 0) {
            for (long long idx = tid(); idx < (long long)j * m; idx += LSDD_WG) {
                int i = (int)(idx % j), c = (int)(idx / j);
                B[i + (long long)c * ldb] -= L[j + (long long)i * ldl] * B[j + (long long)c * ldb];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- Jacobi eigensolver

// Parallel cyclic Jacobi (round-robin ordering) on a symmetric n x n matrix a.
// On return a is diagonal up to the rotation threshold (eigenvalues on the
// diagonal) and v (n x n) holds the eigenvectors as columns (v must be the
// identity, or any orthogonal start, on entry).  A pair is rotated when
// |a_pq| > rel * sqrt(|a_pp a_qq|) and |a_pq| > abs_tol; the sweep loop stops
// after a sweep with no rotation.  LDS scratch: `pairs` (2 * npair ints),
// `cs` (2 * npair doubles), `flag` (1 int) with npair = (n + 1) / 2.
__device__ inline int wg_jacobi(double* a, int lda, int n, double* v, int ldv, int max_sweeps,
                                double rel, double abs_tol, int* pairs, double* cs, int* flag) {
    const int np = n + (n & 1);
    const int npair = np / 2;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid() == 0) *flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; ++rnd) {
            for (int k = tid(); k < npair; k += LSDD_WG) {
                int i0 = k, i1 = np - 1 - k;
                int p = (i0 == 0) ? 0 : 1 + ((i0 - 1 + rnd) % (np - 1));
                int q = (i1 == 0) ? 0 : 1 + ((i1 - 1 + rnd) % (np - 1));
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    double app = a[p + (long long)p * lda], aqq = a[q + (long long)q * lda];
                    double apq = a[p + (long long)q * lda];
                    if (fabs(apq) > abs_tol && fabs(apq) > rel * sqrt(fabs(app * aqq))) {
                        double th = (aqq - app) / (2.0 * apq);
                        double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        *flag = 1;
                    }
                }
                pairs[2 * k] = p;
                pairs[2 * k + 1] = (q < n) ? q : -1;
                cs[2 * k] = c;
                cs[2 * k + 1] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (long long idx = tid(); idx < (long long)npair * n; idx += LSDD_WG) {
                int k = (int)(idx % npair), j = (int)(idx / npair);
                int q = pairs[2 * k + 1];
                double s = cs[2 * k + 1];
                if (q < 0 || s == 0.0) continue;
                int p = pairs[2 * k];
                double c = cs[2 * k];
                double* ap = a + p + (long long)j * lda;
                double* aq = a + q + (long long)j * lda;
                double x = *ap, y = *aq;
                *ap = c * x - s * y;
                *aq = s * x + c * y;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (long long idx = tid(); idx < (long long)npair * n; idx += LSDD_WG) {
                int i = (int)(idx % n), k = (int)(idx / n);
                int q = pairs[2 * k + 1];
                double s = cs[2 * k + 1];
                if (q < 0 || s == 0.0) continue;
                int p = pairs[2 * k];
                double c = cs[2 * k];
                double* ap = a + i + (long long)p * lda;
                double* aq = a + i + (long long)q * lda;
                double x = *ap, y = *aq;
                *ap = c * x - s * y;
                *aq = s * x + c * y;
                double* vp = v + i + (long long)p * ldv;
                double* vq = v + i + (long long)q * ldv;
                x = *vp;
                y = *vq;
                *vp = c * x - s * y;
                *vq = s * x + c * y;
            }
            __syncthreads();
        }
        int any = *flag;
        __syncthreads();
        if (!any) break;
    }
    return sweep;
}

// After wg_jacobi: write eigenvalues ascending into w[n] and the matching
// eigenvectors (columns of v) into vs (n x n, ldvs).  Ties keep index order.
__device__ inline void wg_sort_eig(const double* a, int lda, const double* v, int ldv, int n,
                                   double* w, double* vs, int ldvs, int* rank_scratch) {
    for (int i = tid(); i < n; i += LSDD_WG) {
        double di = a[i + (long long)i * lda];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            double dj = a[j + (long long)j * lda];
            r += (dj < di) || (dj == di && j < i);
        }
        rank_scratch[i] = r;
        w[r] = di;
    }
    __syncthreads();
    for (long long idx = tid(); idx < (long long)n * n; idx += LSDD_WG) {
        int i = (int)(idx % n), j = (int)(idx / n);
        vs[i + (long long)rank_scratch[j] * ldvs] = v[i + (long long)j * ldv];
    }
    __syncthreads();
}

}  // namespace lsdd
