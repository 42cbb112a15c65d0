// Workgroup-cooperative dense linear algebra for the batched local problems.
//
// Every routine is executed by all threads of one workgroup (blockDim.x ==
// LSDD_WG) on one matrix; matrices are column-major with a leading dimension
// and may live in LDS or in global memory (flat addressing).  The routines
// synchronise internally and leave the workgroup synchronised on return.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "consts.hpp"
#include "mgemm.hpp"

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

namespace lsdd {

// ---------------------------------------------------------------- tridiagonal eigensolver

// Householder reduction of the symmetric n x n matrix a (column-major, both
// triangles, ld n) to tridiagonal form T = Q^T A Q.  Outputs d[n], e[n-1],
// tau[n-2]; the Householder vector of step j is stored in a[j+2.., j] (its
// leading entry 1 implicit).  LDS scratch: v, w (n doubles each), red.
__device__ inline void wg_tridiag(double* a, int n, double* d, double* e, double* tau, double* v, double* w,
                                  double* red) {
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        double* x = a + (j + 1) + (long long)j * n;           // a[j+1.., j]
        double s2 = 0.0;
        for (int i = 1 + tid(); i < m; i += LSDD_WG) s2 += x[i] * x[i];
        s2 = wg_sum(s2, red);
        const double alpha = x[0];
        double t = 0.0, beta = alpha;
        if (s2 > 0.0) {
            double nrm = sqrt(alpha * alpha + s2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            const double sc = 1.0 / (alpha - beta);
            for (int i = tid(); i < m; i += LSDD_WG) v[i] = (i == 0) ? 1.0 : x[i] * sc;
        } else {
            for (int i = tid(); i < m; i += LSDD_WG) v[i] = (i == 0) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (tid() == 0) {
            d[j] = a[j + (long long)j * n];
            e[j] = beta;
            tau[j] = t;
        }
        if (t != 0.0) {
            // p = t * A22 v  (A22 = a[j+1.., j+1..])
            double* A22 = a + (j + 1) + (long long)(j + 1) * n;
            for (int i = tid(); i < m; i += LSDD_WG) {
                double s = 0.0;
                for (int k = 0; k < m; ++k) s += A22[i + (long long)k * n] * v[k];
                w[i] = t * s;
            }
            __syncthreads();
            double pv = 0.0;
            for (int i = tid(); i < m; i += LSDD_WG) pv += w[i] * v[i];
            pv = wg_sum(pv, red);
            const double K = 0.5 * t * pv;
            for (int i = tid(); i < m; i += LSDD_WG) w[i] -= K * v[i];
            __syncthreads();
            for (long long idx = tid(); idx < (long long)m * m; idx += LSDD_WG) {
                int i = (int)(idx % m), k = (int)(idx / m);
                A22[i + (long long)k * n] -= v[i] * w[k] + w[i] * v[k];
            }
        }
        // keep the reflector below the subdiagonal
        for (int i = 1 + tid(); i < m; i += LSDD_WG) x[i] = v[i];
        __syncthreads();
    }
    if (tid() == 0) {
        if (n >= 2) {
            d[n - 2] = a[(n - 2) + (long long)(n - 2) * n];
            e[n - 2] = a[(n - 1) + (long long)(n - 2) * n];
        }
        d[n - 1] = a[(n - 1) + (long long)(n - 1) * n];
    }
    __syncthreads();
}

// Number of eigenvalues of the tridiagonal (d, e) smaller than x (Sturm count).
__device__ inline int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
    for (int k = 1; k < n; ++k) {
        q = d[k] - x - e[k - 1] * e[k - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++c;
    }
    return c;
}

// Eigenvalues i0 .. i1-1 (ascending order) of the symmetric tridiagonal (d, e)
// by bisection; the bracket is computed from the whole matrix, so any split of
// the index range gives the same values.
__device__ inline void wg_bisect_range(const double* d, const double* e, int n, double* lam, int i0, int i1,
                                       double* red) {
    double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
    for (int i = tid(); i < n; i += LSDD_WG) {
        double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
        if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
    }
    lo = -wg_max(-lo, red);
    hi = wg_max(hi, red);
    emax2 = wg_max(emax2, red);
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = fmax(2.2250738585072014e-308 * fmax(emax2, 1.0), 1e-300);
    const double atol = 2.0 * 2.220446049250313e-16 * tnorm + 1e-300;
    lo -= atol;
    hi += atol;
    for (int i = i0 + tid(); i < i1; i += LSDD_WG) {
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (a + b);
            if (b - a <= 2.0 * 2.220446049250313e-16 * fmax(fabs(a), fabs(b)) + atol || mid == a || mid == b) break;
            if (sturm_count(d, e, n, mid, pivmin) > i) b = mid;
            else a = mid;
        }
        lam[i] = 0.5 * (a + b);
    }
    __syncthreads();
}

// All eigenvalues of the symmetric tridiagonal (d, e), ascending, by bisection.
__device__ inline void wg_bisect_all(const double* d, const double* e, int n, double* lam, double* red) {
    wg_bisect_range(d, e, n, lam, 0, n, red);
}

// Solve (T - lam I) y = b in place for the tridiagonal (d, e) by Gaussian
// elimination with partial pivoting.  b has stride bs; the upper factor
// scratch u0, u1, u2 (n entries each) has stride S, so the 64 lanes of a wave
// solving 64 systems at once can keep their scratch interleaved (S = 64,
// coalesced) without changing the arithmetic.  The elimination is applied to
// b as the factor is formed (one pass), then back substitution.  Both passes
// load the operands of the next block of TRI_PB rows before working on the
// current block, so a lane's chain of dependent divisions does not wait on
// memory latency or on the completion of its own stores.
constexpr int TRI_PB = 8;

template <int S>
__device__ inline void tri_shift_solve(const double* __restrict__ d, const double* __restrict__ e, int n, double lam,
                                       double* __restrict__ b, int bs, double* __restrict__ u0,
                                       double* __restrict__ u1, double* __restrict__ u2, double tiny) {
    // rows k hold (u0[k], u1[k], u2[k]) on diagonals 0, +1, +2 of U; both pivot
    // cases share one division (the quotient of the smaller by the larger of
    // a0 and the subdiagonal entry)
    double a0 = d[0] - lam, a1 = (n > 1) ? e[0] : 0.0;
    double bk = b[0];
    double E[TRI_PB + 1], D[TRI_PB], B[TRI_PB];
    double En[TRI_PB + 1], Dn[TRI_PB], Bn[TRI_PB];
    auto fetch_fwd = [&](int k0, double (&e_)[TRI_PB + 1], double (&d_)[TRI_PB], double (&b_)[TRI_PB]) {
#pragma unroll
        for (int u = 0; u <= TRI_PB; ++u) e_[u] = (k0 + u < n - 1) ? e[k0 + u] : 0.0;
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            const bool ok = k0 + u < n - 1;
            d_[u] = ok ? d[k0 + u + 1] : 0.0;
            b_[u] = ok ? b[(k0 + u + 1) * bs] : 0.0;
        }
    };
    fetch_fwd(0, E, D, B);
    for (int k0 = 0; k0 < n - 1; k0 += TRI_PB) {
        if (k0 + TRI_PB < n - 1) fetch_fwd(k0 + TRI_PB, En, Dn, Bn);
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            const int k = k0 + u;
            if (k < n - 1) {
                const double sub = E[u];
                const double nd = D[u] - lam;
                const double ns = E[u + 1];           // e[k + 1], 0 past the end
                const bool sw = !(fabs(a0) >= fabs(sub));
                if (!sw && fabs(a0) < tiny) a0 = (a0 >= 0.0 ? tiny : -tiny);
                const double den = sw ? sub : a0;
                const double f = (sw ? a0 : sub) / den;
                u0[k * S] = den;
                u1[k * S] = sw ? nd : a1;
                u2[k * S] = sw ? ns : 0.0;
                const double a0n = sw ? a1 - f * nd : nd - f * a1;
                a1 = sw ? -f * ns : ns;
                a0 = a0n;
                // the same elimination step on b (rows k and k + 1, swapped if pivoted)
                double bn = B[u];
                if (sw) {
                    const double t = bk;
                    bk = bn;
                    bn = t;
                }
                b[k * bs] = bk;
                bk = bn - f * bk;
            }
        }
#pragma unroll
        for (int u = 0; u <= TRI_PB; ++u) E[u] = En[u];
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            D[u] = Dn[u];
            B[u] = Bn[u];
        }
    }
    if (fabs(a0) < tiny) a0 = (a0 >= 0.0 ? tiny : -tiny);
    u0[(n - 1) * S] = a0;
    u1[(n - 1) * S] = 0.0;
    u2[(n - 1) * S] = 0.0;
    b[(n - 1) * bs] = bk;
    // back substitution, rows n-1 .. 0 in blocks of TRI_PB (row k = k1 - u)
    double Y[TRI_PB], P0[TRI_PB], P1[TRI_PB], P2[TRI_PB];
    double Yn[TRI_PB], P0n[TRI_PB], P1n[TRI_PB], P2n[TRI_PB];
    auto fetch_bwd = [&](int k1, double (&y_)[TRI_PB], double (&p0)[TRI_PB], double (&p1)[TRI_PB],
                         double (&p2)[TRI_PB]) {
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            const int k = k1 - u;
            const bool ok = k >= 0;
            y_[u] = ok ? b[k * bs] : 0.0;
            p0[u] = ok ? u0[k * S] : 1.0;
            p1[u] = ok ? u1[k * S] : 0.0;
            p2[u] = ok ? u2[k * S] : 0.0;
        }
    };
    double x1 = 0.0, x2 = 0.0;
    fetch_bwd(n - 1, Y, P0, P1, P2);
    for (int k1 = n - 1; k1 >= 0; k1 -= TRI_PB) {
        if (k1 - TRI_PB >= 0) fetch_bwd(k1 - TRI_PB, Yn, P0n, P1n, P2n);
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            const int k = k1 - u;
            if (k >= 0) {
                double s = Y[u];
                if (k + 1 < n) s -= P1[u] * x1;
                if (k + 2 < n) s -= P2[u] * x2;
                const double xk = s / P0[u];
                b[k * bs] = xk;
                x2 = x1;
                x1 = xk;
            }
        }
#pragma unroll
        for (int u = 0; u < TRI_PB; ++u) {
            Y[u] = Yn[u];
            P0[u] = P0n[u];
            P1[u] = P1n[u];
            P2[u] = P2n[u];
        }
    }
}

// dd[j + t qn] = Q_j . Y_t for the columns Q_j = V[:, q0 + j] (j < qn <= 64) and
// Y_t = V[:, b0 + t] (t < bn <= 64) of the column-major V (ld n): each thread
// accumulates a 4 x 4 block of products over the rows in order.
__device__ inline void wg_block_dots(const double* V, int n, int q0, int qn, int b0, int bn, double* dd) {
    const int ib = tid() & 15, jb = tid() >> 4;
    if (4 * ib >= qn || 4 * jb >= bn) return;
    const double* qp[4];
    const double* yp[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        qp[a] = V + (long long)(q0 + min(4 * ib + a, qn - 1)) * n;
        yp[a] = V + (long long)(b0 + min(4 * jb + a, bn - 1)) * n;
    }
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int k = 0; k < n; ++k) {
        double qv[4], yv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            qv[a] = qp[a][k];
            yv[a] = yp[a][k];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += qv[a] * yv[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (4 * ib + a < qn && 4 * jb + c < bn) dd[(4 * ib + a) + (4 * jb + c) * qn] = acc[a][c];
}

// Y_t -= sum_j dd[j + t qn] Q_j (same columns as wg_block_dots); each thread
// takes 4 rows x 4 members, the sum over j in order.
__device__ inline void wg_block_update(double* V, int n, int q0, int qn, int b0, int bn, const double* dd) {
    const int nr = (n + 3) / 4, nc = (bn + 3) / 4;
    for (int w = tid(); w < nr * nc; w += LSDD_WG) {
        const int r = 4 * (w % nr), c0 = 4 * (w / nr);
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
        for (int j = 0; j < qn; ++j) {
            const double* q = V + (long long)(q0 + j) * n + r;
            double qv[4], dv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                qv[a] = (r + a < n) ? q[a] : 0.0;
                dv[a] = (c0 + a < bn) ? dd[j + (c0 + a) * qn] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] += qv[a] * dv[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (r + a < n && c0 + c < bn) V[(long long)(b0 + c0 + c) * n + r + a] -= acc[a][c];
    }
}

// The same two steps on the FP64 matrix cores (one 64 x 64 tile of Q^T Y with
// K = n; then Y -= Q dd tile by tile down the rows).
__device__ inline void wg_block_dots_mfma(mg::Smem& sm, const double* V, int n, int q0, int qn, int b0, int bn,
                                          double* dd) {
    mg::d4 acc[2][2];
    mg::zero(acc);
    mg::tile_mma<mg::KMAJ, mg::KMAJ>(sm, V + (long long)q0 * n, n, 0, qn, V + (long long)b0 * n, n, 0, bn, 0, n,
                                     acc);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = mg::acc_row(p, v), j = mg::acc_col(q);
                if (i < qn && j < bn) dd[i + j * qn] = acc[p][q][v];
            }
}

__device__ inline void wg_block_update_mfma(mg::Smem& sm, double* V, int n, int q0, int qn, int b0, int bn,
                                            const double* dd) {
    if (bn <= 0) return;   // uniform over the workgroup
    for (int r0 = 0; r0 < n; r0 += mg::T) {
        mg::d4 acc[2][2];
        mg::zero(acc);
        mg::tile_mma<mg::IMAJ, mg::KMAJ>(sm, V + (long long)q0 * n + r0, n, 0, n - r0, dd, qn, 0, bn, 0, qn, acc);
        double old[2][2][4];   // loaded before use, addresses clamped (no conditional loads)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = min(r0 + mg::acc_row(p, v), n - 1), t = min(mg::acc_col(q), bn - 1);
                    old[p][q][v] = V[(long long)(b0 + t) * n + i];
                }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = r0 + mg::acc_row(p, v), t = mg::acc_col(q);
                    if (i < n && t < bn) V[(long long)(b0 + t) * n + i] = old[p][q][v] - acc[p][q][v];
                }
    }
}

// Orthonormalise the batch Y = V[:, b0 .. b0 + bn) by Cholesky QR: with D the
// inverse column norms, D Y^T Y D = L L^T and Y <- Y D L^{-T}.  That is the Q of
// Y = QR, the factor Gram-Schmidt in index order produces, from one product on
// the matrix cores, a 64 x 64 Cholesky in LDS and one triangular solve per row.
// Returns false, with Y unchanged, when a pivot of the unit-diagonal Gram matrix
// falls below 1e-12 (cond(Y D) above about 1e6, where one pass would lose
// orthogonality); the caller then orthogonalises member by member.  dd: 64 x 64
// doubles of global scratch.
__device__ inline bool wg_batch_cholqr(mg::Smem& sm, double* V, int n, int b0, int bn, double* dd) {
    __shared__ int s_ok;
    __shared__ double s_d[64];
    wg_block_dots_mfma(sm, V, n, b0, bn, b0, bn, dd);
    __syncthreads();
    double* G = reinterpret_cast<double*>(&sm);                // bn * bn <= 4096 doubles
    for (int i = tid(); i < bn; i += LSDD_WG) {
        const double g = dd[i + i * bn];
        s_d[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
    }
    if (tid() == 0) s_ok = 1;
    __syncthreads();
    for (int idx = tid(); idx < bn * bn; idx += LSDD_WG) G[idx] = dd[idx] * s_d[idx % bn] * s_d[idx / bn];
    __syncthreads();
    for (int j = 0; j < bn; ++j) {
        const double pjj = G[j + j * bn];
        if (!(pjj > 1e-12)) {
            if (tid() == 0) s_ok = 0;
            break;                                              // same value on every thread
        }
        const double ljj = sqrt(pjj);
        for (int i = j + 1 + tid(); i < bn; i += LSDD_WG) G[i + j * bn] /= ljj;
        __syncthreads();
        const int m = bn - 1 - j;                               // trailing (i, k), j < k <= i
        for (int idx = tid(); idx < m * m; idx += LSDD_WG) {
            const int i = j + 1 + idx % m, k = j + 1 + idx / m;
            if (k <= i) G[i + k * bn] -= G[i + j * bn] * G[k + j * bn];
        }
        if (tid() == 0) G[j + j * bn] = ljj;
        __syncthreads();
    }
    __syncthreads();
    const bool ok = s_ok != 0;
    if (ok) {
        for (int r = tid(); r < n; r += LSDD_WG)
            for (int j = 0; j < bn; ++j) {
                double z = V[(long long)(b0 + j) * n + r] * s_d[j];
                for (int k = 0; k < j; ++k) z -= V[(long long)(b0 + k) * n + r] * G[j + k * bn];
                V[(long long)(b0 + j) * n + r] = z / G[j + j * bn];
            }
    }
    __syncthreads();
    return ok;
}

// Eigenvectors of the tridiagonal (d, e) for the eigenvalues lam[0..kk) by
// inverse iteration.  Eigenvalues closer than 1e-4 * tnorm form a cluster.
// This workgroup handles the single-member clusters with index in [r0, r1)
// and the larger clusters that start there.  Singletons run one per thread
// (threads 0..63).  `ws` holds INVIT_SLOTS * n doubles: the factor scratch
// (u0, u1, u2) and singleton iterates of the 64 solving lanes, interleaved by
// lane.  The members of a larger cluster are processed in batches of up
// to 64: each iteration solves every member's shifted system on its own
// thread, then orthogonalises the batch twice: by block classical Gram-Schmidt
// against the earlier members of the cluster, then within the batch by Cholesky
// QR (with sm; wg_batch_cholqr) or, where that is refused or without sm, by
// Gram-Schmidt in index order, normalising each member.  Every vector is computed the same way
// whatever the range split.  Output V (n x kk, column-major, ld n); `dd` holds
// 64 x 64 batch dots.  LDS: cl_start (kk+1 ints), dots (64).
// sm: LDS staging of the matrix cores for the block Gram-Schmidt steps of
// clusters (NULL: the same steps as register-blocked vector loops).
__device__ inline void wg_inverse_iteration_range(const double* d, const double* e, int n, const double* lam,
                                                  int kk, int r0, int r1, double* V, double* ws, double* dd,
                                                  double tnorm, int* cl_start, double* dots, double* red,
                                                  int* ncl_sh, mg::Smem* sm = nullptr) {
    const double eps = 2.220446049250313e-16;
    const double gaptol = 1e-4 * tnorm;
    if (tid() == 0) {
        int nc = 0;
        for (int i = 0; i < kk; ++i)
            if (i == 0 || lam[i] - lam[i - 1] > gaptol) cl_start[nc++] = i;
        cl_start[nc] = kk;
        *ncl_sh = nc;
    }
    __syncthreads();
    const int ncl = *ncl_sh;
    const double tiny = eps * fmax(tnorm, 1e-300);
    // convergence: from the second solve on, the iterate entering a solve has unit norm,
    // so the norm of the result is the solve's growth 1 / |lambda - shift| along the
    // eigenvector; once it exceeds 1 / (1e-10 ||T||) (shift within 1e-10 ||T|| of an
    // eigenvalue, at least 1e-4 ||T|| from every other cluster) each further solve would
    // shrink the error by at least 1e6, and the iteration stops (at most 4 solves)
    const double grow2 = 1.0 / ((1e-10 * fmax(tnorm, 1e-300)) * (1e-10 * fmax(tnorm, 1e-300)));
    __shared__ int s_conv;
    auto start_value = [&](int i, int k) {
        unsigned h = (unsigned)(k * 2654435761u) ^ (unsigned)(i * 40503u);
        return 1.0 + 0.25 * ((double)(h & 0xffff) / 65536.0 - 0.5);
    };
    // lane-interleaved scratch of the 64 solving threads (lane t: entry k at [64 k + t])
    auto slot_solve = [&](int t, double* b, int bs, double shift) {
        tri_shift_solve<64>(d, e, n, shift, b, bs, ws + t, ws + (long long)64 * n + t, ws + (long long)128 * n + t,
                            tiny);
    };
    // singletons, one per thread
    for (int i = r0 + tid(); tid() < 64 && i < r1; i += 64) {
        int lo = 0, hi = ncl;                          // cluster of i: last start <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cl_start[mid] <= i) lo = mid;
            else hi = mid;
        }
        if (cl_start[lo] != i || cl_start[lo + 1] != i + 1) continue;
        double* y = ws + (long long)192 * n + tid();      // interleaved iterate
        for (int k = 0; k < n; ++k) y[64 * k] = start_value(i, k);
        for (int it = 0; it < 4; ++it) {
            slot_solve(tid(), y, 64, lam[i]);
            double nr = 0.0;
            for (int k = 0; k < n; ++k) nr += y[64 * k] * y[64 * k];
            const bool conv = it >= 1 && nr >= grow2;
            nr = 1.0 / sqrt(nr);
            for (int k = 0; k < n; ++k) y[64 * k] *= nr;
            if (conv) break;
        }
        double* out = V + (long long)i * n;
        for (int k = 0; k < n; ++k) out[k] = y[64 * k];
    }
    __syncthreads();
    // clusters, in batches of up to 64 members
    for (int c = 0; c < ncl; ++c) {
        const int c0 = cl_start[c], c1 = cl_start[c + 1];
        if (c1 - c0 == 1 || c0 < r0 || c0 >= r1) continue;
        for (int b0 = c0; b0 < c1; b0 += 64) {
            const int bn = min(64, c1 - b0), np = b0 - c0;
            for (long long idx = tid(); idx < (long long)bn * n; idx += LSDD_WG) {
                const int i = b0 + (int)(idx / n), k = (int)(idx % n);
                V[(long long)i * n + k] = start_value(i, k);
            }
            __syncthreads();
            for (int it = 0; it < 4; ++it) {
                if (tid() == 0) s_conv = 1;
                __syncthreads();
                if (tid() < bn) {
                    double* y = V + (long long)(b0 + tid()) * n;
                    slot_solve(tid(), y, 1, lam[b0 + tid()] + (b0 + tid() - c0) * 2.0 * tiny);
                    if (it >= 1) {
                        double nr = 0.0;
                        for (int k = 0; k < n; ++k) nr += y[k] * y[k];
                        if (!(nr >= grow2)) s_conv = 0;
                    }
                }
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    // against the earlier members of the cluster (in chunks of 64 members)
                    for (int q0 = c0; q0 < b0; q0 += 64) {
                        const int qn = min(64, b0 - q0);
                        if (sm) {
                            wg_block_dots_mfma(*sm, V, n, q0, qn, b0, bn, dd);
                            __syncthreads();
                            wg_block_update_mfma(*sm, V, n, q0, qn, b0, bn, dd);
                        } else {
                            wg_block_dots(V, n, q0, qn, b0, bn, dd);
                            __syncthreads();
                            wg_block_update(V, n, q0, qn, b0, bn, dd);
                        }
                        __syncthreads();
                    }
                    // within the batch: Cholesky QR where the batch is well enough
                    // conditioned, else in index order, each member normalised before use
                    if (sm && wg_batch_cholqr(*sm, V, n, b0, bn, dd)) continue;
                    for (int t = 0; t < bn; ++t) {
                        double* y = V + (long long)(b0 + t) * n;
                        if (t > 0) {
                            for (int s0 = tid() >> 6; s0 < t; s0 += LSDD_WG / 64) {
                                const double* q = V + (long long)(b0 + s0) * n;
                                double s = 0.0;
                                for (int k = tid() & 63; k < n; k += 64) s += q[k] * y[k];
                                s = wave_sum(s);
                                if ((tid() & 63) == 0) dots[s0] = s;
                            }
                            __syncthreads();
                            for (int k = tid(); k < n; k += LSDD_WG) {
                                double s = 0.0;
                                for (int s0 = 0; s0 < t; ++s0) s += V[(long long)(b0 + s0) * n + k] * dots[s0];
                                y[k] -= s;
                            }
                            __syncthreads();
                        }
                        double nr = 0.0;
                        for (int k = tid(); k < n; k += LSDD_WG) nr += y[k] * y[k];
                        nr = wg_sum(nr, red);
                        const double sc = 1.0 / sqrt(nr);
                        for (int k = tid(); k < n; k += LSDD_WG) y[k] *= sc;
                        __syncthreads();
                    }
                }
                const int conv = s_conv;
                __syncthreads();                  // every thread has read the flag before it is reset
                if (it >= 1 && conv) break;
            }
        }
    }
}

// All kk eigenvectors in one workgroup; `ws` holds INVIT_SLOTS * n doubles of
// interleaved scratch followed by 64 x 64 doubles of batch dots.
__device__ inline void wg_inverse_iteration(const double* d, const double* e, int n, const double* lam, int kk,
                                            double* V, double* ws, double tnorm, int* cl_start, double* dots,
                                            double* red, int* ncl_sh) {
    wg_inverse_iteration_range(d, e, n, lam, kk, 0, kk, V, ws, ws + (long long)INVIT_SLOTS * n, tnorm, cl_start,
                               dots, red, ncl_sh);
}

// V <- Q V with Q = H_0 ... H_{n-3} from wg_tridiag (reflectors in a, tau).
__device__ inline void wg_tridiag_backtransform(const double* a, int n, const double* tau, double* V, int kk,
                                                double* vbuf, double* dots) {
    for (int j = n - 3; j >= 0; --j) {
        const double t = tau[j];
        if (t == 0.0) continue;
        const int m = n - j - 1;
        for (int i = tid(); i < m; i += LSDD_WG) vbuf[i] = (i == 0) ? 1.0 : a[(j + 1 + i) + (long long)j * n];
        __syncthreads();
        for (int c = tid(); c < kk; c += LSDD_WG) {
            const double* col = V + (long long)c * n + j + 1;
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += vbuf[i] * col[i];
            dots[c] = t * s;
        }
        __syncthreads();
        for (long long idx = tid(); idx < (long long)m * kk; idx += LSDD_WG) {
            int i = (int)(idx % m), c = (int)(idx / m);
            V[(long long)c * n + j + 1 + i] -= dots[c] * vbuf[i];
        }
        __syncthreads();
    }
}

}  // namespace lsdd
