// Batched, tiled FP64 dense kernels (see batched.hpp).  Grid layout of every
// launch: blockIdx.y = view index, blockIdx.x = tile job inside that view;
// jobs past a view's own job count exit at once (views have different sizes).
//
// The factorisations are blocked with 64 x 64 tiles: the diagonal tile work
// (unblocked Cholesky, triangular substitution) runs in LDS and registers,
// every update of the trailing matrix runs on the FP64 matrix cores through
// the tile contraction of mgemm.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <stdexcept>
#include <string>
#include <type_traits>

#include "batched.hpp"
#include "mgemm.hpp"

namespace lsdd {

namespace {

constexpr int TB = 64;       // tile edge of the blocked algorithms
constexpr int OB = 4;        // tiles per panel of the delayed trailing updates (K = 256)
constexpr int TT = 32;       // tile edge of the transpose
constexpr int NT = 256;

constexpr int NTP = 1024;   // threads of the pivoted-Cholesky panel kernel (one workgroup per matrix)
__device__ inline int t_id() { return (int)threadIdx.x; }
__device__ inline double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int ntiles(int n) { return (n + TB - 1) / TB; }

// 64 x 64 tile (rows r0.., cols c0..) into LDS, zero outside the view; if
// `unit_pad`, padded diagonal entries are 1 (a padded triangular factor).
__device__ inline void ld_tile64(double (*t)[TB + 1], const double* a, const View& v, int r0, int c0,
                                 bool unit_pad = false) {
    for (int idx = t_id(); idx < TB * TB; idx += NT) {
        int i = idx % TB, j = idx / TB;
        int r = r0 + i, c = c0 + j;
        double x = (r < v.rows && c < v.cols) ? a[v.off + r + (int64_t)c * v.ld] : 0.0;
        if (unit_pad && i == j && !(r < v.rows && c < v.cols)) x = 1.0;
        t[i][j] = x;
    }
}

// ---------------------------------------------------------------- substitution in registers
//
// 64 right-hand sides at once: thread t works on vector t / 4 and holds its
// entries sub, sub + 4, ..., sub + 60 (sub = t % 4) in x[16]; the four lanes
// of a vector are adjacent, so pivots are passed by lane shuffles.

// L x = b (L lower, LDS), first nb rows
__device__ inline void fwd_subst(const double (*L)[TB + 1], double (&x)[16], int nb) {
    const int sub = t_id() & 3, base = (t_id() & 63) & ~3;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        if (i < nb) {
            double xi = x[i >> 2] / L[i][i];
            xi = __shfl(xi, base | (i & 3), 64);
            if (sub == (i & 3)) x[i >> 2] = xi;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (4 * q + sub > i) x[q] -= L[4 * q + sub][i] * xi;
        }
    }
}

// L^T x = b (L lower, LDS), first nb rows
__device__ inline void bwd_subst(const double (*L)[TB + 1], double (&x)[16], int nb) {
    const int sub = t_id() & 3, base = (t_id() & 63) & ~3;
#pragma unroll
    for (int i = TB - 1; i >= 0; --i) {
        if (i < nb) {
            double xi = x[i >> 2] / L[i][i];
            xi = __shfl(xi, base | (i & 3), 64);
            if (sub == (i & 3)) x[i >> 2] = xi;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (4 * q + sub < i) x[q] -= L[i][4 * q + sub] * xi;
        }
    }
}

// ---------------------------------------------------------------- Cholesky

// unblocked Cholesky of diagonal tile kb by one wave: lane i holds row i of the
// tile in registers; at column j the pivot is broadcast by a lane shuffle and
// the new column L[:, j] through LDS.  minpiv[view] tracks the smallest pivot
// (a non-positive or NaN pivot is replaced by 1 so the factorisation runs to
// the end; the caller reads minpiv)
__global__ void __launch_bounds__(64) k_potrf_diag(double* base, const View* views, int kb, double* minpiv) {
    __shared__ double col[TB];
    const View v = views[blockIdx.y];
    const int n = v.rows;
    if (kb * TB >= n) return;
    const int r0 = kb * TB, nb = min(TB, n - r0);
    const int i = t_id();
    double x[TB];
    // every lane loads a full row of the block first (row and column clamped into
    // the block, so the 64 loads are unconditional and in flight together), then
    // keeps its lower part (identity rows past the block end)
    const int ic = min(i, nb - 1);
#pragma unroll
    for (int k = 0; k < TB; ++k) x[k] = base[v.off + (r0 + ic) + (int64_t)(r0 + min(k, nb - 1)) * v.ld];
#pragma unroll
    for (int k = 0; k < TB; ++k) x[k] = (i < nb && k <= i) ? x[k] : (k == i ? 1.0 : 0.0);
    double dmin = INFINITY;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
        if (j < nb) {
            double dj = 1.0;
            if (i == j) {
                const double d = x[j];
                dmin = (d == d) ? d : -1.0;
                dj = d > 0.0 ? sqrt(d) : 1.0;
                x[j] = dj;
            }
            dj = __shfl(dj, j, 64);
            if (i > j) x[j] /= dj;
            col[i] = i > j ? x[j] : 0.0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = j + 1; k < TB; ++k)
                if (i >= k) x[k] -= x[j] * col[k];
            __builtin_amdgcn_wave_barrier();
        }
    }
    dmin = wave_min(dmin);
    if (i < nb) {
#pragma unroll
        for (int k = 0; k < TB; ++k)
            if (k <= i) base[v.off + (r0 + i) + (int64_t)(r0 + k) * v.ld] = x[k];
    }
    if (i == 0) minpiv[blockIdx.y] = (kb == 0) ? dmin : fmin(minpiv[blockIdx.y], dmin);
}

// L_ib,kb = A_ib,kb L_kk^{-T}, ib = kb + 1 + blockIdx.x: each row solves
// L_kk x^T = a^T (forward substitution)
__global__ void __launch_bounds__(NT) k_potrf_panel(double* base, const View* views, int kb) {
    __shared__ double L[TB][TB + 1];
    const View v = views[blockIdx.y];
    const int n = v.rows;
    const int nt = ntiles(n);
    const int ib = kb + 1 + (int)blockIdx.x;
    if (ib >= nt) return;
    const int nb = min(TB, n - kb * TB);
    ld_tile64(L, base, v, kb * TB, kb * TB, true);
    __syncthreads();
    const int r = ib * TB + t_id() / 4, sub = t_id() & 3;
    double x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = kb * TB + 4 * q + sub;
        x[q] = (r < n && 4 * q + sub < nb) ? base[v.off + r + (int64_t)c * v.ld] : 0.0;
    }
    fwd_subst(L, x, nb);
    if (r < n) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = kb * TB + 4 * q + sub;
            if (4 * q + sub < nb) base[v.off + r + (int64_t)c * v.ld] = x[q];
        }
    }
}

// A_ib,jb -= sum over column tiles k in [kt0, kt1) of L_ib,k L_jb,k^T, for the
// lower tiles jb in [jt0, jt1), ib >= jb (matrix cores; K up to OB tiles)
__global__ void __launch_bounds__(NT) k_potrf_update(double* base, const View* views, int kt0, int kt1, int jt0,
                                                     int jt1, const int32_t* skip = nullptr) {
    __shared__ mg::Smem sm;
    if (skip && skip[blockIdx.y]) return;
    const View v = views[blockIdx.y];
    const int n = v.rows;
    const int nt = ntiles(n);
    const int K = min(kt1 * TB, n) - kt0 * TB;
    if (K <= 0) return;
    int t = (int)blockIdx.x, jb = jt0;
    const int jend = min(jt1, nt);
    while (jb < jend && t >= nt - jb) {
        t -= nt - jb;
        ++jb;
    }
    if (jb >= jend) return;
    const int ib = jb + t;
    const double* pan = base + v.off + (int64_t)(kt0 * TB) * v.ld;    // column tiles kt0 ..
    mg::d4 acc[2][2];
    mg::zero(acc);
    mg::tile_mma<mg::IMAJ, mg::IMAJ>(sm, pan, v.ld, ib * TB, n, pan, v.ld, jb * TB, n, 0, K, acc);
    // the 16 old entries are loaded before any is used (addresses clamped into the
    // matrix, so no load is conditional and none waits for the previous one)
    double old[2][2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = min(ib * TB + mg::acc_row(p, e), n - 1), c = min(jb * TB + mg::acc_col(q), n - 1);
                old[p][q][e] = base[v.off + r + (int64_t)c * v.ld];
            }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = mg::acc_row(p, e), j = mg::acc_col(q);
                const int r = ib * TB + i, c = jb * TB + j;
                if (r < n && c < n && (ib != jb || i >= j))
                    base[v.off + r + (int64_t)c * v.ld] = old[p][q][e] - acc[p][q][e];
            }
}

// The trailing update of a panel group on 128 x 128 tiles: A[r, c] -= sum over the
// group's columns k of L[r, k] L[c, k] for r >= c >= jt0 TB (lower triangle only).
// Used where the trailing block spans several 128-row blocks.
__global__ void __launch_bounds__(NT, 2) k_potrf_update2(double* base, const View* views, int kt0, int kt1, int jt0,
                                                         const int32_t* skip = nullptr) {
    __shared__ mg::Smem128 sm;
    if (skip && skip[blockIdx.y]) return;
    const View v = views[blockIdx.y];
    const int n = v.rows;
    const int K = min(kt1 * TB, n) - kt0 * TB;
    const int r00 = jt0 * TB;
    if (K <= 0 || r00 >= n) return;
    const int m2 = (n - r00 + mg::T2 - 1) / mg::T2;
    int job = (int)blockIdx.x;
    if (job >= m2 * (m2 + 1) / 2) return;
    int J = 0;
    while (job >= m2 - J) {
        job -= m2 - J;
        ++J;
    }
    const int I = J + job;
    const int rb = r00 + I * mg::T2, cb = r00 + J * mg::T2;
    const double* pan = base + v.off + (int64_t)(kt0 * TB) * v.ld;
    mg::d4 acc[4][4];
    mg::zero(acc);
    mg::tile_mma128<mg::IMAJ, mg::IMAJ>(sm, pan, v.ld, rb, n, pan, v.ld, cb, n, 0, K, acc);
    // per block row: its 16 old entries loaded first (addresses clamped), then updated
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double old[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = min(rb + mg::acc_row2(p, e), n - 1), c = min(cb + mg::acc_col2(q), n - 1);
                old[q][e] = base[v.off + r + (int64_t)c * v.ld];
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rb + mg::acc_row2(p, e), c = cb + mg::acc_col2(q);
                if (r < n && c < n && r >= c) base[v.off + r + (int64_t)c * v.ld] = old[q][e] - acc[p][q][e];
            }
    }
}

// ---------------------------------------------------------------- pivoted Cholesky of a trailing block

// Largest value over [j, n) of d by one workgroup of NTH threads; among equal values
// the one with the lowest key (key[i], or i without keys).  rv, ri: NTH / 64 LDS slots.
template <int NTH>
__device__ inline void wg_argmax(const double* d, const int32_t* key, int j, int n, double* rv, int* ri, double& bv,
                                 int& bi) {
    auto kf = [key](int i) { return key ? key[i] : i; };
    auto better = [&](double xv, int xi, double yv, int yi) {   // (xv, xi) before (yv, yi)
        return xi >= 0 && (yi < 0 || xv > yv || (xv == yv && kf(xi) < kf(yi)));
    };
    bv = -INFINITY;
    bi = -1;
    for (int i = j + t_id(); i < n; i += NTH) {
        const double x = d[i];
        if (better(x, i, bv, bi)) { bv = x; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if ((t_id() & 63) == 0) { rv[t_id() >> 6] = bv; ri[t_id() >> 6] = bi; }
    __syncthreads();
    bv = rv[0];
    bi = ri[0];
    for (int w = 1; w < NTH / 64; ++w)
        if (better(rv[w], ri[w], bv, bi)) { bv = rv[w]; bi = ri[w]; }
    __syncthreads();
}

// Columns [kb TB, kb TB + TB) of the diagonally pivoted Cholesky of the trailing
// block of view b (indices lead[b] .. m-1 of the square view, lower triangle).
// Left-looking inside the panel: the trailing matrix holds the updates of the
// earlier panels only, the panel's own earlier columns are applied per column.
// The pivot is the largest remaining diagonal entry; it is swapped into place
// symmetrically across the whole view (row segment left of it, diagonal, the
// column below), so the leading block keeps its position and the coupling rows
// follow their indices.  The factorisation stops when the largest remaining
// diagonal entry is at most tol[b]: rank[b] is then the number of eliminated
// indices and done[b] is set.  diag: per-view scratch of the remaining diagonal.
// perm (optional, at diag_off like diag): perm[i] is the trailing index whose
// row and column sit at trailing position i; among equal diagonal entries the
// pivot is then the lowest original index (without perm: the lowest position).
__global__ void __launch_bounds__(NTP) k_pstrf_panel(double* base, const View* views, const int32_t* lead, int kb,
                                                     const double* tol, const int64_t* diag_off, double* diag,
                                                     int32_t* perm, int32_t* rank, int32_t* done) {
    __shared__ double rv[NTP / 64];
    __shared__ int ri[NTP / 64];
    __shared__ double s_p[TB];
    if (done[blockIdx.y]) return;
    const View v = views[blockIdx.y];
    const int nw = lead[blockIdx.y];
    const int m = v.rows, ng = m - nw;
    const int64_t ld = v.ld;
    double* M = base + v.off;
    double* D = diag + diag_off[blockIdx.y];
    const double tl = tol[blockIdx.y];
    const int j0 = kb * TB;
    if (j0 >= ng) {
        if (t_id() == 0) { rank[blockIdx.y] = ng; done[blockIdx.y] = 1; }
        return;
    }
    const int j1 = min(j0 + TB, ng);
    int32_t* Pm = perm ? perm + diag_off[blockIdx.y] : nullptr;
    for (int i = j0 + t_id(); i < ng; i += NTP) D[i] = M[(nw + i) + (int64_t)(nw + i) * ld];
    if (Pm && kb == 0)
        for (int i = t_id(); i < ng; i += NTP) Pm[i] = i;
    __syncthreads();
    for (int j = j0; j < j1; ++j) {
        double bv;
        int bi;
        wg_argmax<NTP>(D, Pm, j, ng, rv, ri, bv, bi);
        if (!(bv > tl)) {
            if (t_id() == 0) { rank[blockIdx.y] = j; done[blockIdx.y] = 1; }
            return;
        }
        const int J = nw + j;
        if (bi != j) {
            const int Q = nw + bi;
            for (int q = t_id(); q < m; q += NTP) {
                if (q < J) {
                    const double a = M[J + (int64_t)q * ld];
                    M[J + (int64_t)q * ld] = M[Q + (int64_t)q * ld];
                    M[Q + (int64_t)q * ld] = a;
                } else if (q == J) {
                    const double a = M[J + (int64_t)J * ld];
                    M[J + (int64_t)J * ld] = M[Q + (int64_t)Q * ld];
                    M[Q + (int64_t)Q * ld] = a;
                    const double dd = D[j];
                    D[j] = D[bi];
                    D[bi] = dd;
                    if (Pm) {
                        const int32_t pp = Pm[j];
                        Pm[j] = Pm[bi];
                        Pm[bi] = pp;
                    }
                } else if (q < Q) {
                    const double a = M[q + (int64_t)J * ld];
                    M[q + (int64_t)J * ld] = M[Q + (int64_t)q * ld];
                    M[Q + (int64_t)q * ld] = a;
                } else if (q > Q) {
                    const double a = M[q + (int64_t)J * ld];
                    M[q + (int64_t)J * ld] = M[q + (int64_t)Q * ld];
                    M[q + (int64_t)Q * ld] = a;
                }
            }
            __syncthreads();
        }
        // the pivot row's entries in the panel's earlier columns, staged once
        for (int k = j0 + t_id(); k < j; k += NTP) s_p[k - j0] = M[J + (int64_t)(nw + k) * ld];
        __syncthreads();
        const double ljj = sqrt(D[j]);
        const double inv = 1.0 / ljj;
        // column j below the pivot, left-looking over the panel's earlier columns in
        // four independent partial sums
        for (int i = j + 1 + t_id(); i < ng; i += NTP) {
            const double* mi = M + (nw + i);
            double c0 = mi[(int64_t)J * ld], c1 = 0.0, c2 = 0.0, c3 = 0.0;
            int k = j0;
            for (; k + 4 <= j; k += 4) {
                c0 -= mi[(int64_t)(nw + k) * ld] * s_p[k - j0];
                c1 -= mi[(int64_t)(nw + k + 1) * ld] * s_p[k + 1 - j0];
                c2 -= mi[(int64_t)(nw + k + 2) * ld] * s_p[k + 2 - j0];
                c3 -= mi[(int64_t)(nw + k + 3) * ld] * s_p[k + 3 - j0];
            }
            for (; k < j; ++k) c0 -= mi[(int64_t)(nw + k) * ld] * s_p[k - j0];
            const double c = ((c0 + c1) + (c2 + c3)) * inv;
            M[(nw + i) + (int64_t)J * ld] = c;
            D[i] -= c * c;
        }
        __syncthreads();
        if (t_id() == 0) M[J + (int64_t)J * ld] = ljj;
        __syncthreads();
    }
    if (t_id() == 0) {
        rank[blockIdx.y] = j1;
        if (j1 == ng) done[blockIdx.y] = 1;
    }
}

// ---------------------------------------------------------------- triangular solves

// step s of L X = B (forward, kb = s) or L^T X = B (backward, kb = nt-1-s):
// solve the diagonal tile for column tile jc = blockIdx.x of B.  lower_b: B is
// lower triangular (forward only), so column tiles jc > kb are still zero.
__global__ void __launch_bounds__(NT) k_trsm_diag(const double* lbase, const View* lv, double* bbase, const View* bv,
                                                  int s, int trans, int lower_b) {
    __shared__ double L[TB][TB + 1];
    const View l = lv[blockIdx.y], b = bv[blockIdx.y];
    const int n = l.rows;
    const int nt = ntiles(n);
    if (s >= nt) return;
    const int kb = trans ? nt - 1 - s : s;
    const int jc = (int)blockIdx.x;
    if (jc * TB >= b.cols || (lower_b && jc > kb)) return;
    const int nb = min(TB, n - kb * TB);
    ld_tile64(L, lbase, l, kb * TB, kb * TB, true);
    __syncthreads();
    const int c = jc * TB + t_id() / 4, sub = t_id() & 3;
    double x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = kb * TB + 4 * q + sub;
        x[q] = (c < b.cols && 4 * q + sub < nb) ? bbase[b.off + r + (int64_t)c * b.ld] : 0.0;
    }
    if (!trans) fwd_subst(L, x, nb);
    else bwd_subst(L, x, nb);
    if (c < b.cols) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = kb * TB + 4 * q + sub;
            if (4 * q + sub < nb) bbase[b.off + r + (int64_t)c * b.ld] = x[q];
        }
    }
}

// forward: B_ib -= sum_{k in [kt0, kt1)} L_ib,k X_k for the row tiles ib in
// [it0, it1) (lower_b: column tiles jc < kt1 only); backward (step s, kb =
// nt-1-s, it0/it1/kt0/kt1 unused): B_ib -= L_kb,ib^T X_kb for ib < kb
__global__ void __launch_bounds__(NT) k_trsm_update(const double* lbase, const View* lv, double* bbase, const View* bv,
                                                    int kt0, int kt1, int it0, int it1, int s, int trans,
                                                    int lower_b) {
    __shared__ mg::Smem sm;
    const View l = lv[blockIdx.y], b = bv[blockIdx.y];
    const int n = l.rows;
    const int nt = ntiles(n);
    int nct = ntiles(b.cols);
    int row0, nrow, k0, K;
    if (!trans) {
        k0 = kt0;
        K = min(kt1 * TB, n) - kt0 * TB;
        row0 = it0;
        nrow = min(it1, nt) - it0;
        if (lower_b) nct = min(nct, kt1);
    } else {
        if (s >= nt) return;
        k0 = nt - 1 - s;
        K = min(TB, n - k0 * TB);
        row0 = 0;
        nrow = k0;
    }
    if (K <= 0 || nrow <= 0) return;
    const int job = (int)blockIdx.x;
    if (job >= nrow * nct) return;
    const int ib = row0 + job % nrow;
    const int jc = job / nrow;
    const double* xk = bbase + b.off + k0 * TB;                       // X_k0..: element (k, j) at xk[k + j ld]
    mg::d4 acc[2][2];
    mg::zero(acc);
    if (!trans) {
        const double* lp = lbase + l.off + (int64_t)(k0 * TB) * l.ld;  // L[:, k0..]: (k, i) at lp[i + k ld]
        mg::tile_mma<mg::IMAJ, mg::KMAJ>(sm, lp, l.ld, ib * TB, n, xk, b.ld, jc * TB, b.cols, 0, K, acc);
    } else {
        const double* lp = lbase + l.off + k0 * TB;                    // L[kb, :]: (k, i) at lp[k + i ld]
        mg::tile_mma<mg::KMAJ, mg::KMAJ>(sm, lp, l.ld, ib * TB, n, xk, b.ld, jc * TB, b.cols, 0, K, acc);
    }
    double old[2][2][4];   // loaded before use, addresses clamped (no conditional loads)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = min(ib * TB + mg::acc_row(p, e), b.rows - 1), c = min(jc * TB + mg::acc_col(q), b.cols - 1);
                old[p][q][e] = bbase[b.off + r + (int64_t)c * b.ld];
            }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = ib * TB + mg::acc_row(p, e), c = jc * TB + mg::acc_col(q);
                if (r < b.rows && c < b.cols) bbase[b.off + r + (int64_t)c * b.ld] = old[p][q][e] - acc[p][q][e];
            }
}

// Forward trailing update on 128 x 128 tiles: B[r, c] -= sum_{k in [kt0, kt1) tiles}
// L[r, k] X[k, c] for rows r >= kt1 TB and columns c < ccap (lower_b: ccap = kt1 TB).
__global__ void __launch_bounds__(NT, 2) k_trsm_update2(const double* lbase, const View* lv, double* bbase,
                                                        const View* bv, int kt0, int kt1, int lower_b) {
    __shared__ mg::Smem128 sm;
    const View l = lv[blockIdx.y], b = bv[blockIdx.y];
    const int n = l.rows;
    const int K = min(kt1 * TB, n) - kt0 * TB;
    const int r00 = kt1 * TB;
    const int ccap = lower_b ? min(b.cols, kt1 * TB) : b.cols;
    if (K <= 0 || r00 >= n || ccap <= 0) return;
    const int nr2 = (n - r00 + mg::T2 - 1) / mg::T2, nc2 = (ccap + mg::T2 - 1) / mg::T2;
    const int job = (int)blockIdx.x;
    if (job >= nr2 * nc2) return;
    const int rb = r00 + (job % nr2) * mg::T2, cb = (job / nr2) * mg::T2;
    const double* lp = lbase + l.off + (int64_t)(kt0 * TB) * l.ld;   // L[:, kt0..]: (k, i) at lp[i + k ld]
    const double* xk = bbase + b.off + kt0 * TB;                      // X rows kt0..: (k, j) at xk[k + j ld]
    mg::d4 acc[4][4];
    mg::zero(acc);
    mg::tile_mma128<mg::IMAJ, mg::KMAJ>(sm, lp, l.ld, rb, n, xk, b.ld, cb, ccap, 0, K, acc);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double old[4][4];   // loaded first, addresses clamped (no conditional loads)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = min(rb + mg::acc_row2(p, e), b.rows - 1), c = min(cb + mg::acc_col2(q), ccap - 1);
                old[q][e] = bbase[b.off + r + (int64_t)c * b.ld];
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rb + mg::acc_row2(p, e), c = cb + mg::acc_col2(q);
                if (r < b.rows && c < ccap) bbase[b.off + r + (int64_t)c * b.ld] = old[q][e] - acc[p][q][e];
            }
    }
}

// ---------------------------------------------------------------- C = beta C_in - alpha A^T B

template <bool F32>
__global__ void __launch_bounds__(NT) k_gemm_tn(const double* abase, const View* av, const double* bbase,
                                                const View* bv, const double* cinbase, const View* civ, double beta,
                                                double* coutbase, const View* cov, double alpha, int tri_k, int sym) {
    __shared__ typename std::conditional<F32, mg::Smem32, mg::Smem>::type sm;
    const View a = av[blockIdx.y], b = bv[blockIdx.y], co = cov[blockIdx.y];
    const int mt = ntiles(co.rows), ntt = ntiles(co.cols);
    int it, jt;
    int job = (int)blockIdx.x;
    if (sym) {
        if (job >= mt * (mt + 1) / 2) return;
        jt = 0;
        while (job >= mt - jt) { job -= mt - jt; ++jt; }
        it = jt + job;
    } else {
        if (job >= mt * ntt) return;
        it = job % mt;
        jt = job / mt;
    }
    const int kbeg = tri_k ? max(it, jt) * TB : 0;
    const View ci = civ[blockIdx.y];
    // C_in entries are loaded for the whole tile before any is used (addresses clamped
    // into C, so the loads are unconditional and issued back to back)
    double cin[2][2][4];
    auto load_cin = [&](auto row_of) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = min(it * TB + row_of(p, e), co.rows - 1), c = min(jt * TB + mg::acc_col(q), co.cols - 1);
                    cin[p][q][e] = beta != 0.0 ? cinbase[ci.off + r + (int64_t)c * ci.ld] : 0.0;
                }
    };
    auto put = [&](int r, int c, double s, double old) {
        if (r < co.rows && c < co.cols) {
            double x = -alpha * s;
            if (beta != 0.0) x += beta * old;
            coutbase[co.off + r + (int64_t)c * co.ld] = x;
            if (sym && it != jt) coutbase[co.off + c + (int64_t)r * co.ld] = x;
        }
    };
    if constexpr (F32) {
        mg::f4 acc[2][2];
        mg::zero32(acc);
        mg::tile_mma32<mg::KMAJ, mg::KMAJ>(sm, abase + a.off, a.ld, it * TB, a.cols, bbase + b.off, b.ld, jt * TB,
                                           b.cols, kbeg, a.rows, acc);
        if (beta != 0.0) load_cin([](int p, int e) { return mg::acc_row32(p, e); });
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    put(it * TB + mg::acc_row32(p, e), jt * TB + mg::acc_col(q), (double)acc[p][q][e], cin[p][q][e]);
    } else {
        mg::d4 acc[2][2];
        mg::zero(acc);
        mg::tile_mma<mg::KMAJ, mg::KMAJ>(sm, abase + a.off, a.ld, it * TB, a.cols, bbase + b.off, b.ld, jt * TB,
                                         b.cols, kbeg, a.rows, acc);
        if (beta != 0.0) load_cin([](int p, int e) { return mg::acc_row(p, e); });
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    put(it * TB + mg::acc_row(p, e), jt * TB + mg::acc_col(q), acc[p][q][e], cin[p][q][e]);
    }
}

// C = beta C_in - alpha A^T B on 128 x 128 tiles (FP64), as k_gemm_tn<false>
__global__ void __launch_bounds__(NT, 2) k_gemm_tn2(const double* abase, const View* av, const double* bbase,
                                                    const View* bv, const double* cinbase, const View* civ,
                                                    double beta, double* coutbase, const View* cov, double alpha,
                                                    int tri_k, int sym) {
    __shared__ mg::Smem128 sm;
    const View a = av[blockIdx.y], b = bv[blockIdx.y], co = cov[blockIdx.y];
    const int mt = (co.rows + mg::T2 - 1) / mg::T2, ntt = (co.cols + mg::T2 - 1) / mg::T2;
    int it, jt;
    int job = (int)blockIdx.x;
    if (sym) {
        if (job >= mt * (mt + 1) / 2) return;
        jt = 0;
        while (job >= mt - jt) {
            job -= mt - jt;
            ++jt;
        }
        it = jt + job;
    } else {
        if (job >= mt * ntt) return;
        it = job % mt;
        jt = job / mt;
    }
    const int kbeg = tri_k ? max(it, jt) * mg::T2 : 0;
    const View ci = civ[blockIdx.y];
    mg::d4 acc[4][4];
    mg::zero(acc);
    mg::tile_mma128<mg::KMAJ, mg::KMAJ>(sm, abase + a.off, a.ld, it * mg::T2, a.cols, bbase + b.off, b.ld,
                                        jt * mg::T2, b.cols, kbeg, a.rows, acc);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double old[4][4];   // C_in loaded first, addresses clamped (no conditional loads)
        if (beta != 0.0) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = min(it * mg::T2 + mg::acc_row2(p, e), co.rows - 1);
                    const int c = min(jt * mg::T2 + mg::acc_col2(q), co.cols - 1);
                    old[q][e] = cinbase[ci.off + r + (int64_t)c * ci.ld];
                }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = it * mg::T2 + mg::acc_row2(p, e), c = jt * mg::T2 + mg::acc_col2(q);
                if (r < co.rows && c < co.cols) {
                    double x = -alpha * acc[p][q][e];
                    if (beta != 0.0) x += beta * old[q][e];
                    coutbase[co.off + r + (int64_t)c * co.ld] = x;
                    if (sym && it != jt) coutbase[co.off + c + (int64_t)r * co.ld] = x;
                }
            }
    }
}

// ---------------------------------------------------------------- transpose

__global__ void __launch_bounds__(NT) k_transpose(double* base, const View* views) {
    __shared__ double P[TT][TT + 1];
    __shared__ double Q[TT][TT + 1];
    const View v = views[blockIdx.y];
    const int nt = (v.rows + TT - 1) / TT;
    int t = (int)blockIdx.x;
    if (t >= nt * (nt + 1) / 2) return;
    int jt = 0;
    while (t > jt) { t -= jt + 1; ++jt; }
    const int it = t;   // it <= jt
    for (int idx = t_id(); idx < TT * TT; idx += NT) {
        int i = idx % TT, j = idx / TT;
        int r = it * TT + i, c = jt * TT + j;
        P[i][j] = (r < v.rows && c < v.cols) ? base[v.off + r + (int64_t)c * v.ld] : 0.0;
        int r2 = jt * TT + i, c2 = it * TT + j;
        Q[i][j] = (r2 < v.rows && c2 < v.cols) ? base[v.off + r2 + (int64_t)c2 * v.ld] : 0.0;
    }
    __syncthreads();
    for (int idx = t_id(); idx < TT * TT; idx += NT) {
        int i = idx % TT, j = idx / TT;
        int r = it * TT + i, c = jt * TT + j;
        if (r < v.rows && c < v.cols) base[v.off + r + (int64_t)c * v.ld] = Q[j][i];
        int r2 = jt * TT + i, c2 = it * TT + j;
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

static int max_tiles(const std::vector<View>& v, bool rows, int tb = TB) {
    int m = 0;
    for (const View& x : v) m = std::max(m, ((rows ? x.rows : x.cols) + tb - 1) / tb);
    return m;
}

void Batched::potrf(double* base, const std::vector<View>& a, double* d_minpiv) {
    if (a.empty()) return;
    View* dv = put(0, a);
    const unsigned nm = (unsigned)a.size();
    const int nt = max_tiles(a, true);
    // right-looking over panels of OB tile columns: inside a panel the updates
    // reach the panel's own columns (K = one tile), the rest of the trailing
    // matrix is updated once per panel with K = OB tiles
    for (int p0 = 0; p0 < nt; p0 += OB) {
        const int p1 = std::min(p0 + OB, nt);
        for (int kb = p0; kb < p1; ++kb) {
            hipLaunchKernelGGL(k_potrf_diag, dim3(1, nm), dim3(64), 0, st, base, dv, kb, d_minpiv);
            const int below = nt - kb - 1;
            if (below <= 0) continue;
            hipLaunchKernelGGL(k_potrf_panel, dim3(below, nm), dim3(NT), 0, st, base, dv, kb);
            int64_t jobs = 0;
            for (int jb = kb + 1; jb < p1; ++jb) jobs += nt - jb;
            if (jobs > 0)
                hipLaunchKernelGGL(k_potrf_update, dim3((unsigned)jobs, nm), dim3(NT), 0, st, base, dv, kb, kb + 1,
                                   kb + 1, p1);
        }
        if (p1 < nt) {
            const int64_t m = nt - p1;
            if (m >= 4) {      // at least two 128-row blocks: the 128 x 128 tiles
                const int64_t m2 = (m + 1) / 2;
                hipLaunchKernelGGL(k_potrf_update2, dim3((unsigned)(m2 * (m2 + 1) / 2), nm), dim3(NT), 0, st, base,
                                   dv, p0, p1, p1);
            } else {
                hipLaunchKernelGGL(k_potrf_update, dim3((unsigned)(m * (m + 1) / 2), nm), dim3(NT), 0, st, base, dv,
                                   p0, p1, p1, nt);
            }
        }
    }
    chk(hipGetLastError(), "batched potrf");
}

void Batched::pstrf_trailing(double* base, const std::vector<View>& a, const std::vector<int32_t>& lead,
                             const double* d_tol, std::vector<int32_t>& rank, int32_t* d_perm) {
    rank.assign(a.size(), 0);
    if (a.empty()) return;
    const size_t nv = a.size();
    std::vector<View> g(nv);
    std::vector<int64_t> doff(nv + 1, 0);
    int max_ng = 0;
    for (size_t b = 0; b < nv; ++b) {
        const int ng = a[b].rows - lead[b];
        if (ng < 0 || a[b].rows != a[b].cols) throw std::runtime_error("batched pstrf: bad view");
        g[b] = View{a[b].off + lead[b] + (int64_t)lead[b] * a[b].ld, a[b].ld, ng, ng, 0};
        doff[b + 1] = doff[b] + ng;
        max_ng = std::max(max_ng, ng);
    }
    View* dv = put(0, a);
    View* dg = put(1, g);
    int32_t* d_lead = (int32_t*)alloc(ctx, nv * sizeof(int32_t));
    int64_t* d_doff = (int64_t*)alloc(ctx, (nv + 1) * sizeof(int64_t));
    double* d_diag = (double*)alloc(ctx, std::max<int64_t>(doff[nv], 1) * sizeof(double));
    int32_t* d_state = (int32_t*)alloc(ctx, 2 * nv * sizeof(int32_t));
    chk(hipMemcpyAsync(d_lead, lead.data(), nv * sizeof(int32_t), hipMemcpyHostToDevice, st), "pstrf upload");
    chk(hipMemcpyAsync(d_doff, doff.data(), (nv + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), "pstrf upload");
    chk(hipMemsetAsync(d_state, 0, 2 * nv * sizeof(int32_t), st), "pstrf state");
    int32_t* d_rank = d_state;
    int32_t* d_done = d_state + nv;
    const unsigned nm = (unsigned)nv;
    const int nt = (max_ng + TB - 1) / TB;
    for (int kb = 0; kb < nt; ++kb) {
        hipLaunchKernelGGL(k_pstrf_panel, dim3(1, nm), dim3(NTP), 0, st, base, dv, d_lead, kb, d_tol, d_doff, d_diag,
                           d_perm, d_rank, d_done);
        const int64_t m = nt - kb - 1;
        if (m >= 4) {
            const int64_t m2 = (m + 1) / 2;
            hipLaunchKernelGGL(k_potrf_update2, dim3((unsigned)(m2 * (m2 + 1) / 2), nm), dim3(NT), 0, st, base, dg,
                               kb, kb + 1, kb + 1, (const int32_t*)d_done);
        } else if (m > 0) {
            hipLaunchKernelGGL(k_potrf_update, dim3((unsigned)(m * (m + 1) / 2), nm), dim3(NT), 0, st, base, dg, kb,
                               kb + 1, kb + 1, nt, (const int32_t*)d_done);
        }
    }
    chk(hipGetLastError(), "batched pstrf");
    chk(hipMemcpyAsync(rank.data(), d_rank, nv * sizeof(int32_t), hipMemcpyDeviceToHost, st), "pstrf rank");
    chk(hipStreamSynchronize(st), "pstrf sync");
    for (void* p : {(void*)d_lead, (void*)d_doff, (void*)d_diag, (void*)d_state}) release(ctx, p);
}

void Batched::trsm(const double* lbase, const std::vector<View>& l, double* bbase, const std::vector<View>& b,
                   bool trans, bool lower_b) {
    if (l.empty()) return;
    if (trans && lower_b) throw std::runtime_error("batched trsm: lower_b applies to forward solves only");
    View* d1 = put(0, l);
    View* d2 = put(1, b);
    const unsigned nm = (unsigned)l.size();
    const int nt = max_tiles(l, true);
    const int nct = max_tiles(b, false);
    if (nct == 0) return;
    if (trans) {
        // backward solves (few right-hand sides here): one tile step at a time
        for (int s = 0; s < nt; ++s) {
            hipLaunchKernelGGL(k_trsm_diag, dim3(nct, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, s, 1, 0);
            const int jobs = (nt - 1 - s) * nct;
            if (jobs > 0)
                hipLaunchKernelGGL(k_trsm_update, dim3(jobs, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, 0, 0, 0, 0,
                                   s, 1, 0);
        }
    } else {
        // forward over panels of OB tile rows: updates inside the panel with K =
        // one tile, the rows below once per panel with K = OB tiles
        for (int p0 = 0; p0 < nt; p0 += OB) {
            const int p1 = std::min(p0 + OB, nt);
            for (int kb = p0; kb < p1; ++kb) {
                hipLaunchKernelGGL(k_trsm_diag, dim3(nct, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, kb, 0,
                                   lower_b ? 1 : 0);
                const int cols = lower_b ? std::min(nct, kb + 1) : nct;
                const int jobs = (p1 - kb - 1) * cols;
                if (jobs > 0)
                    hipLaunchKernelGGL(k_trsm_update, dim3(jobs, nm), dim3(NT), 0, st, lbase, d1, bbase, d2, kb,
                                       kb + 1, kb + 1, p1, 0, 0, lower_b ? 1 : 0);
            }
            if (p1 < nt) {
                const int cols = lower_b ? std::min(nct, p1) : nct;
                if (nt - p1 >= 4 && cols >= 2) {   // 128 x 128 tiles where the block is large enough
                    const int64_t jobs = (int64_t)((nt - p1 + 1) / 2) * ((cols + 1) / 2);
                    hipLaunchKernelGGL(k_trsm_update2, dim3((unsigned)jobs, nm), dim3(NT), 0, st, lbase, d1, bbase, d2,
                                       p0, p1, lower_b ? 1 : 0);
                } else {
                    const int64_t jobs = (int64_t)(nt - p1) * cols;
                    hipLaunchKernelGGL(k_trsm_update, dim3((unsigned)jobs, nm), dim3(NT), 0, st, lbase, d1, bbase, d2,
                                       p0, p1, p1, nt, 0, 0, lower_b ? 1 : 0);
                }
            }
        }
    }
    chk(hipGetLastError(), "batched trsm");
}

void Batched::gemm_tn(const double* abase, const std::vector<View>& a, const double* bbase, const std::vector<View>& b,
                      const double* cinbase, const std::vector<View>& cin, double beta, double* coutbase,
                      const std::vector<View>& cout, double alpha, bool tri_k, bool sym, bool f32) {
    if (a.empty()) return;
    if (sym && beta != 0.0) throw std::runtime_error("batched gemm_tn: sym needs beta = 0");
    View* d1 = put(0, a);
    View* d2 = put(1, b);
    View* d3 = put(2, cout);
    View* d4 = beta != 0.0 ? put(3, cin) : d3;
    const unsigned nm = (unsigned)a.size();
    int64_t mt = 0;
    for (const View& x : cout) {
        const int64_t r = (x.rows + TB - 1) / TB, c = (x.cols + TB - 1) / TB;
        mt = std::max(mt, sym ? r * (r + 1) / 2 : r * c);
    }
    if (mt == 0) return;
    if (mt > INT32_MAX) throw std::runtime_error("batched gemm_tn: too many tiles");
    int64_t mt2 = 0, big = 0;
    for (const View& x : cout) {
        const int64_t r = (x.rows + 127) / 128, c = (x.cols + 127) / 128;
        mt2 = std::max(mt2, sym ? r * (r + 1) / 2 : r * c);
        big = std::max<int64_t>(big, std::min(x.rows, x.cols));
    }
    if (!f32 && big >= 256) {   // 128 x 128 tiles once the outputs span several of them
        hipLaunchKernelGGL(k_gemm_tn2, dim3((unsigned)mt2, nm), dim3(NT), 0, st, abase, d1, bbase, d2, cinbase, d4,
                           beta, coutbase, d3, alpha, tri_k ? 1 : 0, sym ? 1 : 0);
        chk(hipGetLastError(), "batched gemm_tn");
        return;
    }
    if (f32)
        hipLaunchKernelGGL(k_gemm_tn<true>, dim3((unsigned)mt, nm), dim3(NT), 0, st, abase, d1, bbase, d2, cinbase, d4,
                           beta, coutbase, d3, alpha, tri_k ? 1 : 0, sym ? 1 : 0);
    else
        hipLaunchKernelGGL(k_gemm_tn<false>, dim3((unsigned)mt, nm), dim3(NT), 0, st, abase, d1, bbase, d2, cinbase,
                           d4, beta, coutbase, d3, alpha, tri_k ? 1 : 0, sym ? 1 : 0);
    chk(hipGetLastError(), "batched gemm_tn");
}

void Batched::transpose(double* base, const std::vector<View>& a) {
    if (a.empty()) return;
    View* d1 = put(0, a);
    const unsigned nm = (unsigned)a.size();
    const int nt = max_tiles(a, true, TT);
    hipLaunchKernelGGL(k_transpose, dim3(nt * (nt + 1) / 2, nm), dim3(NT), 0, st, base, d1);
    chk(hipGetLastError(), "batched transpose");
}

}  // namespace lsdd
