// Block (multi right-hand side) cycle kernels and the segmented PCG of the
// batched solve, for CDNA4 (gfx950).
//
// Block vectors interleave NRB = 8 right-hand sides per DOF, so each matrix,
// inverse or interpolation entry read from HBM is used for all of them: the
// cycle's bytes per right-hand side drop by up to 8x against separate solves.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <stdexcept>
#include <type_traits>

#include "blk.hpp"
#include "kernels.hpp"
#include "dense.hpp"
#include "symv.hpp"

namespace lsdd {

namespace {

constexpr int WG = LSDD_WG;
constexpr int NB = NRB;

// compute units of the current device (queried once per device)
int device_cu_count() {
    static int count[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!count[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        count[dev] = n;
    }
    return count[dev];
}

inline unsigned grid_for(int64_t n, int per_block = WG) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65535LL * 64) g = 65535LL * 64;
    return (unsigned)g;
}

// ---------------------------------------------------------------- CSR
// L lanes per row; lane = (nonzero slot, right-hand side): L / NB nonzeros per step.
template <typename T, int L>
__global__ void __launch_bounds__(WG) k_csr_resid_rows_b(int64_t nrows, const int32_t* rows, const int64_t* rowptr,
                                                         const int32_t* col, const T* val, const T* x, const T* r,
                                                         T* out, int x_zero, const int64_t* scoff) {
    constexpr int NS = L / NB;
    const int lane = tid() & (L - 1), k = lane & (NB - 1), slot = lane / NB;
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t t = ((int64_t)blockIdx.x * WG + tid()) / L; t < nrows; t += stride) {
        const int32_t p = rows[t];   // < 0: masked entry, out = 0
        T s = 0;
        if (!x_zero && p >= 0) {
            const int64_t q1 = rowptr[p + 1], cb = scoff ? scoff[p] - rowptr[p] : 0;
#pragma unroll 4
            for (int64_t q = rowptr[p] + slot; q < q1; q += NS) s += val[q] * x[(int64_t)col[cb + q] * NB + k];
        }
        for (int off = L / 2; off >= NB; off >>= 1) s += __shfl_xor(s, off, L);
        if (slot == 0) out[t * NB + k] = p >= 0 ? r[(int64_t)p * NB + k] - s : (T)0;
    }
}

// L lanes per row (4, 8 or 16); lane = nonzero slot holding all NB right-hand
// sides: it reads its entries' values and columns once and each gathered row of
// x with 16-byte loads (two entries in flight; past the row end the index is
// clamped to the last entry and the value zeroed, so the loads need no branch).
// The NB sums are reduced over the L lanes by a transposing butterfly (4 + 2 + 1
// exchanges over 8 lanes leave lane l with right-hand side l; 4 + 2 over 4 lanes
// leave it with 2l and 2l + 1), then by plain exchanges over the remaining lane
// bits; the order is fixed.
template <typename T>
struct Row16 {
    using V = double2;
};
template <>
struct Row16<float> {
    using V = float4;
};

template <typename T>
__device__ inline void load_xrow(const T* p, T (&v)[NB]) {
    using V = typename Row16<T>::V;
    constexpr int W = 16 / sizeof(T);
    const V* pv = reinterpret_cast<const V*>(p);
#pragma unroll
    for (int u = 0; u < NB / W; ++u) {
        const V t = pv[u];
        const T* tt = reinterpret_cast<const T*>(&t);
#pragma unroll
        for (int c = 0; c < W; ++c) v[u * W + c] = tt[c];
    }
}

template <typename T, int L>
__device__ inline void slot_row_sums(int64_t q0, int64_t q1, int lane, const int32_t* col, int64_t cb, const T* val,
                                     const T* x, T (&s)[NB]) {
    const int nit = (int)((q1 - q0 + L - 1) / L);
    for (int it = 0; it < nit; it += 2) {
        const int64_t qa = q0 + lane + (int64_t)it * L, qb = qa + L;
        const int64_t qac = qa < q1 ? qa : q1 - 1, qbc = qb < q1 ? qb : q1 - 1;
        const T va = val[qac], vb = val[qbc];
        const int32_t ca = col[cb + qac], cc = col[cb + qbc];
        T xa[NB], xb[NB];
        load_xrow(x + (int64_t)ca * NB, xa);
        load_xrow(x + (int64_t)cc * NB, xb);
        const T wa = qa < q1 ? va : (T)0, wb = qb < q1 ? vb : (T)0;
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] += wa * xa[k];
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] += wb * xb[k];
    }
}

// one butterfly step: lanes paired across lane bit `o` swap halves of their
// first 2 C values and keep the half selected by that bit
template <typename T, int L, int C>
__device__ inline void slot_fold(T (&s)[NB], int lane, int o) {
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const T send = hi ? s[i] : s[i + C], keep = hi ? s[i + C] : s[i];
        s[i] = keep + __shfl_xor(send, o, L);
    }
}

// B = min(L, NB) lanes split the NB sums: afterwards lane l < B holds right-hand
// sides (NB / B) l + i in s[i], i < NB / B, summed over all L lanes of the row
template <typename T, int L>
__device__ inline void slot_reduce(T (&s)[NB], int lane) {
    static_assert(NB == 8 && L >= 4 && L <= 64, "butterfly laid out for 8 right-hand sides");
    constexpr int B = L < NB ? L : NB;
    slot_fold<T, L, 4>(s, lane, B / 2);
    slot_fold<T, L, 2>(s, lane, B / 4);
    if constexpr (B == 8) slot_fold<T, L, 1>(s, lane, 1);
#pragma unroll
    for (int off = 8; off < L; off <<= 1) s[0] += __shfl_xor(s[0], off, L);
}

template <typename T, int L>
__global__ void __launch_bounds__(WG) k_csr_resid_rows_s(int64_t nrows, const int32_t* rows, const int64_t* rowptr,
                                                         const int32_t* col, const T* val, const T* x, const T* r,
                                                         T* out, int x_zero, const int64_t* scoff) {
    const int lane = tid() & (L - 1);
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t t = ((int64_t)blockIdx.x * WG + tid()) / L; t < nrows; t += stride) {
        const int32_t p = rows[t];   // < 0: masked entry, out = 0
        T s[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] = 0;
        if (!x_zero && p >= 0)
            slot_row_sums<T, L>(rowptr[p], rowptr[p + 1], lane, col, scoff ? scoff[p] - rowptr[p] : 0, val, x, s);
        slot_reduce<T, L>(s, lane);
        constexpr int PL = L < NB ? NB / L : 1;   // right-hand sides per writing lane
        if (lane * PL < NB)
#pragma unroll
            for (int i = 0; i < PL; ++i) {
                const int k = lane * PL + i;
                out[t * NB + k] = p >= 0 ? r[(int64_t)p * NB + k] - s[i] : (T)0;
            }
    }
}

template <typename T, int L>
__global__ void __launch_bounds__(WG) k_csr_spmv_s(int64_t n, const int64_t* rowptr, const int32_t* col,
                                                   const T* val, const T* x, T* y, const T* r_minus,
                                                   const int64_t* scoff) {
    const int lane = tid() & (L - 1);
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t p = ((int64_t)blockIdx.x * WG + tid()) / L; p < n; p += stride) {
        T s[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] = 0;
        slot_row_sums<T, L>(rowptr[p], rowptr[p + 1], lane, col, scoff ? scoff[p] - rowptr[p] : 0, val, x, s);
        slot_reduce<T, L>(s, lane);
        constexpr int PL = L < NB ? NB / L : 1;
        if (lane * PL < NB)
#pragma unroll
            for (int i = 0; i < PL; ++i) {
                const int k = lane * PL + i;
                y[p * NB + k] = r_minus ? r_minus[p * NB + k] - s[i] : s[i];
            }
    }
}

template <typename T, int L>
__global__ void __launch_bounds__(WG) k_csr_spmv_b(int64_t n, const int64_t* rowptr, const int32_t* col,
                                                   const T* val, const T* x, T* y, const T* r_minus,
                                                   const int64_t* scoff) {
    constexpr int NS = L / NB;
    const int lane = tid() & (L - 1), k = lane & (NB - 1), slot = lane / NB;
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t p = ((int64_t)blockIdx.x * WG + tid()) / L; p < n; p += stride) {
        const int64_t q1 = rowptr[p + 1], cb = scoff ? scoff[p] - rowptr[p] : 0;
        T s = 0;
#pragma unroll 4
        for (int64_t q = rowptr[p] + slot; q < q1; q += NS) s += val[q] * x[(int64_t)col[cb + q] * NB + k];
        for (int off = L / 2; off >= NB; off >>= 1) s += __shfl_xor(s, off, L);
        if (slot == 0) y[p * NB + k] = r_minus ? r_minus[p * NB + k] - s : s;
    }
}

// ---------------------------------------------------------------- subdomain product
// Same work items and partial layout as the single-vector kernel, with NB-wide
// entries.  Each tile is staged once in LDS (rows padded to 65 entries, so both
// row-wise and column-wise reads are free of bank conflicts); the right-hand-side
// entries are wave-uniform and come through the scalar cache.  Every lane works on
// all NB right-hand sides, so one LDS read of a tile entry feeds NB products: for
// the row part wave w takes the tile's columns 16w .. 16w + 15 with lane = row
// (accumulated over the item's tiles in registers), for the column part its rows
// 16w .. 16w + 15 with lane = column; the four waves' partial sums are added in
// wave order through LDS (per tile for the column part, once per item for the
// row part).  The next tile is prefetched into registers (non-temporal loads: the
// tiles stream once per application) while the current one is used.
template <typename T>
__global__ void __launch_bounds__(WG) k_sub_symv_b(const int32_t* items, const int64_t* sub_off,
                                                   const int64_t* tp_off, const T* __restrict__ tiles,
                                                   const T* __restrict__ rloc, const int64_t* scr_off,
                                                   T* __restrict__ scr, int chl) {
    __shared__ T s_t[64 * 65];
    const int s = items[3 * blockIdx.x];
    const int I = items[3 * blockIdx.x + 1];
    const int ch = items[3 * blockIdx.x + 2];
    const int64_t o = sub_off[s];
    const int m = (int)(sub_off[s + 1] - o);
    const int nt = (m + 63) >> 6;
    const int J0 = ch * chl;
    const int nJ = min(chl, I + 1 - J0);
    const int lane = tid() & 63, w = tid() >> 6;
    // wave-uniform quarter of the tile; the right-hand-side entries it multiplies are
    // read at wave-uniform addresses (scalar loads), clamped to the subdomain's last
    // row: the tiles are zero past |Omega|, so a clamped entry adds nothing
    const int wu = __builtin_amdgcn_readfirstlane(w);
    T* part = scr + scr_off[s] * NB;
    T* colpart = part + symv_rowpart_off(nt, chl) * 64 * NB;
    const T* row0 = tiles + tp_off[s] + (int64_t)I * (I + 1) / 2 * 4096;
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(row0 + (int64_t)J0 * 4096 + i * WG + tid());
    static_assert(WG == 256, "four waves split a tile's columns (row part) and rows (column part)");
    const int q0 = 16 * wu;
    const T* xI = rloc + o * NB;
    T ar[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) ar[k] = 0;
    for (int jj = 0; jj < nJ; ++jj) {
        const int J = J0 + jj;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = i * WG + tid();
            s_t[(e >> 6) * 65 + (e & 63)] = v[i];
        }
        __syncthreads();
        if (jj + 1 < nJ) {
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(row0 + (int64_t)(J + 1) * 4096 + i * WG + tid());
        }
        // row part: lane = row, this wave's 16 columns, all NB right-hand sides
        {
            const T* tr = s_t + lane * 65 + q0;
#pragma unroll 4
            for (int cc = 0; cc < 16; ++cc) {
                const T a = tr[cc];
                const T* xc = xI + (int64_t)min(J * 64 + q0 + cc, m - 1) * NB;
#pragma unroll
                for (int k = 0; k < NB; ++k) ar[k] += a * xc[k];
            }
        }
        if (J < I) {
            // column part: lane = column, this wave's 16 rows; the four row quarters
            // are summed in order through the (then free) tile buffer
            T ac[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) ac[k] = 0;
#pragma unroll 4
            for (int rr = 0; rr < 16; ++rr) {
                const T a = s_t[(q0 + rr) * 65 + lane];
                const T* xr = xI + (int64_t)min(I * 64 + q0 + rr, m - 1) * NB;
#pragma unroll
                for (int k = 0; k < NB; ++k) ac[k] += a * xr[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NB; ++k) s_t[(w * 64 + lane) * NB + k] = ac[k];
            __syncthreads();
            const int c = tid() >> 2, k0 = 2 * (tid() & 3);
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s0 += s_t[(q * 64 + c) * NB + k0];
                s1 += s_t[(q * 64 + c) * NB + k0 + 1];
            }
            T* cp = colpart + (((int64_t)I * (I - 1) / 2 + J) * 64 + c) * NB + k0;
            cp[0] = s0;
            cp[1] = s1;
        }
    }
    // row part: the four column quarters summed in order
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) s_t[(w * 64 + lane) * NB + k] = ar[k];
    __syncthreads();
    const int r = tid() >> 2, k0 = 2 * (tid() & 3);
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s0 += s_t[(q * 64 + r) * NB + k0];
        s1 += s_t[(q * 64 + r) * NB + k0 + 1];
    }
    T* rp = part + ((symv_rowpart_off(I, chl) + ch) * 64 + r) * NB + k0;
    rp[0] = s0;
    rp[1] = s1;
}

// FL threads per DOF sum fixed strided subsets of its partials (all NB
// right-hand sides at once); the FL sums are added in ascending order.
template <typename T, int FL>
__global__ void __launch_bounds__(WG) k_sub_finalize_b(int64_t r0, int64_t r1, const int32_t* pos_sub,
                                                       const int64_t* sub_off, const int64_t* scr_off, const T* scr,
                                                       const int32_t* sub_dofs, T* x, int accumulate, int chl) {
    constexpr int ND = WG / FL;
    __shared__ T s_y[FL][ND][NB];
    const int dl = tid() % ND, j = tid() / ND;
    const int64_t t = r0 + (int64_t)blockIdx.x * ND + dl;
    T y[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) y[q] = 0;
    if (t < r1) {
        const int s = pos_sub[t];
        const int64_t o = sub_off[s];
        const int c = (int)(t - o);
        const int nt = (int)((sub_off[s + 1] - o + 63) >> 6);
        const int J = c >> 6, l = c & 63;
        const T* part = scr + (scr_off[s] + symv_rowpart_off(J, chl) * 64 + l) * NB;
        const T* colpart = scr + (scr_off[s] + symv_rowpart_off(nt, chl) * 64 + l) * NB;
        const int nch = (J + chl) / chl;
        const int K = nch + (nt - 1 - J);
        for (int k = j; k < K; k += FL) {
            const T* src;
            if (k < nch) {
                src = part + (int64_t)k * 64 * NB;
            } else {
                const int64_t I = J + 1 + (k - nch);
                src = colpart + (I * (I - 1) / 2 + J) * 64 * NB;
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) y[q] += src[q];
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) s_y[j][dl][q] = y[q];
    __syncthreads();
    if (j < NB && t < r1) {
        T v = s_y[0][dl][j];
        for (int q = 1; q < FL; ++q) v += s_y[q][dl][j];
        const int64_t d = sub_dofs ? (int64_t)sub_dofs[t] : t;   // < 0: masked entry
        if (d >= 0) x[d * NB + j] = accumulate ? x[d * NB + j] + v : v;
    }
}

// ---------------------------------------------------------------- transfers
// Restriction rc[coff_i + s] = sum_a Z_i[a, s] t[omega_i[a]] for all right-hand
// sides: work item = (aggregate, 16 columns); t on omega_i is staged in LDS in
// chunks of 256 rows, each wave takes 4 columns, lanes stride the rows.
template <typename T>
__global__ void __launch_bounds__(WG) k_restrict_b(const int32_t* items, const int64_t* agg_ptr,
                                                   const int32_t* agg_dofs, const int64_t* zoff, const int32_t* k,
                                                   const int64_t* coff, const T* Zc, const T* t, T* rc) {
    __shared__ T s_t[256 * NB];
    const int ag = items[2 * blockIdx.x], s0 = items[2 * blockIdx.x + 1];
    const int kk = k[ag];
    const int64_t a0 = agg_ptr[ag];
    const int nw = (int)(agg_ptr[ag + 1] - a0);
    const int lane = tid() & 63, w = tid() >> 6;
    const T* z = Zc + zoff[ag];
    T acc[4][NB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[i][q] = 0;
    for (int c0 = 0; c0 < nw; c0 += 256) {
        const int cn = min(256, nw - c0);
        __syncthreads();
        if (tid() < cn) {
            const T* src = t + (int64_t)agg_dofs[a0 + c0 + tid()] * NB;
#pragma unroll
            for (int q = 0; q < NB; ++q) s_t[tid() * NB + q] = src[q];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = s0 + w + 4 * i;
            if (s < kk) {
                const T* col = z + (int64_t)s * nw + c0;
                for (int a = lane; a < cn; a += 64) {
                    const T zz = col[a];
#pragma unroll
                    for (int q = 0; q < NB; ++q) acc[i][q] += zz * s_t[a * NB + q];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int s = s0 + w + 4 * i;
        T mine = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            T v = acc[i][q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == q) mine = v;
        }
        if (s < kk && lane < NB) rc[(coff[ag] + s) * NB + lane] = mine;
    }
}

// Prolongation x[omega_i[a]] += sum_s Z_i[a, s] ec[coff_i + s]: work item =
// (aggregate, 256 rows); thread per row, ec staged in LDS in chunks of 256 modes.
template <typename T>
__global__ void __launch_bounds__(WG) k_prolong_b(const int32_t* items, const int64_t* agg_ptr,
                                                  const int32_t* agg_dofs, const int64_t* zoff, const int32_t* k,
                                                  const int64_t* coff, const T* Zc, const T* ec, T* x) {
    __shared__ T s_e[256 * NB];
    const int ag = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
    const int kk = k[ag];
    const int64_t a0 = agg_ptr[ag];
    const int nw = (int)(agg_ptr[ag + 1] - a0);
    const int a = r0 + tid();
    const T* z = Zc + zoff[ag] + a;
    T acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = 0;
    for (int sc = 0; sc < kk; sc += 256) {
        const int sn = min(256, kk - sc);
        __syncthreads();
        for (int e = tid(); e < sn * NB; e += WG) s_e[e] = ec[(coff[ag] + sc) * NB + e];
        __syncthreads();
        if (a < nw) {
            for (int s = 0; s < sn; ++s) {
                const T zz = z[(int64_t)(sc + s) * nw];
#pragma unroll
                for (int q = 0; q < NB; ++q) acc[q] += zz * s_e[s * NB + q];
            }
        }
    }
    if (a < nw) {
        T* dst = x + (int64_t)agg_dofs[a0 + a] * NB;
#pragma unroll
        for (int q = 0; q < NB; ++q) dst[q] += acc[q];
    }
}

// ---------------------------------------------------------------- small overlaps
// Overlaps with |Omega| <= SMALL_M: the inverse is stored as its packed lower
// triangle (entry (i, j), j <= i, at i (i + 1) / 2 + j), staged in LDS by one
// wave per subdomain; lane i forms y_i = sum_j (A_Omega^{-1})_{ij} r_j over all j in
// ascending order (fixed order) and adds it to x (entries with a negative DOF are
// skipped): subdomains of one colour are disjoint, so the update needs no partial
// sums.  The LDS is sized by the launch's largest overlap (max_m), so small
// overlaps leave room for more waves per CU.  FACT: the packed triangle is a
// lower-triangular factor X and the local solve is X^T (X r): lane i first forms
// w_i = sum_{j <= i} X_ij r_j into LDS, then y_i = sum_{j >= i} X_ji w_j.
//
// Persistent waves: wave b takes subdomains b, b + gridDim.x, ...; the triangle and
// right-hand sides of the next subdomain are loaded into registers while the
// current one is computed from LDS, so the loads of one subdomain overlap the
// arithmetic of the previous one.  Loads go in groups of 8 per lane, a group only
// where the subdomain reaches it; inside a group a slot past the end re-reads the
// last entry (same cache line) and is never stored.
template <typename T, int NR, bool FACT>
__global__ void __launch_bounds__(64) k_small_sub(int32_t s0, int32_t n_sub, const int64_t* sub_off,
                                                  const int32_t* sub_dofs, const int64_t* pk_off, const T* pk,
                                                  const T* rloc, T* x, int max_m) {
    constexpr int PG = 8;
    constexpr int PMAX = ((SMALL_M * (SMALL_M + 1) / 2 + 63) / 64 + PG - 1) / PG * PG;   // triangle loads per lane
    constexpr int XMAX = ((SMALL_M * NR + 63) / 64 + PG - 1) / PG * PG;                   // rhs loads per lane
    extern __shared__ __align__(16) unsigned char s_small[];
    T* s_a = reinterpret_cast<T*>(s_small);
    T* s_x = s_a + max_m * (max_m + 1) / 2;
    T* s_w = s_x + max_m * NR;
    const int lane = tid();
    T ra[PMAX], rx[XMAX];
    int64_t o_n = 0;
    int m_n = 0;
    auto fetch = [&](int sb) {
        o_n = sub_off[s0 + sb];
        m_n = (int)(sub_off[s0 + sb + 1] - o_n);
        const T* A = pk + pk_off[s0 + sb];
        const int np = m_n * (m_n + 1) / 2, nx = m_n * NR;
        const T* r = rloc + o_n * NR;
#pragma unroll
        for (int g = 0; g < PMAX; g += PG)
            if (g * 64 < np) {
#pragma unroll
                for (int u = g; u < g + PG; ++u) ra[u] = A[min(lane + 64 * u, np - 1)];
            }
#pragma unroll
        for (int g = 0; g < XMAX; g += PG)
            if (g * 64 < nx) {
#pragma unroll
                for (int u = g; u < g + PG; ++u) rx[u] = r[min(lane + 64 * u, nx - 1)];
            }
    };
    // the factor form keeps its sums in FP64 (FP32 storage): its two products
    // would otherwise each add FP32 rounding to an ill-conditioned local solve
    using Acc = typename std::conditional<FACT, double, T>::type;
    int sb = blockIdx.x;
    if (sb < n_sub) fetch(sb);
    for (; sb < n_sub; sb += gridDim.x) {
        const int64_t o = o_n;
        const int m = m_n;
        const int np = m * (m + 1) / 2;
        __syncthreads();                                   // the previous subdomain's reads of LDS are done
#pragma unroll
        for (int u = 0; u < PMAX; ++u)
            if (lane + 64 * u < np) s_a[lane + 64 * u] = ra[u];
#pragma unroll
        for (int u = 0; u < XMAX; ++u)
            if (lane + 64 * u < m * NR) s_x[lane + 64 * u] = rx[u];
        __syncthreads();
        // this subdomain's DOFs and their current x, loaded ahead of the prefetch so
        // that waiting for them does not wait for it (lanes >= m read a valid entry and
        // store nothing; a masked entry reads x[0]); the colour's subdomains are
        // disjoint, so no other wave writes these x during the launch
        const int32_t d = m > 0 ? sub_dofs[o + min(lane, m - 1)] : -1;
        T xo[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) xo[k] = x[(int64_t)max(d, 0) * NR + k];
        if (sb + (int)gridDim.x < n_sub) fetch(sb + gridDim.x);   // in flight during the arithmetic below
        if (FACT) {
            if (lane < m) {
                const int i = lane;
                const int ri = i * (i + 1) / 2;
                Acc wv[NR];
#pragma unroll
                for (int k = 0; k < NR; ++k) wv[k] = 0;
                for (int j = 0; j <= i; ++j) {
                    const Acc a = s_a[ri + j];
#pragma unroll
                    for (int k = 0; k < NR; ++k) wv[k] += a * (Acc)s_x[j * NR + k];
                }
#pragma unroll
                for (int k = 0; k < NR; ++k) s_w[i * NR + k] = (T)wv[k];
            }
            __syncthreads();
        }
        if (lane < m) {
            const int i = lane;
            const int ri = i * (i + 1) / 2;
            Acc y[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) y[k] = 0;
            if (FACT) {
                for (int j = i; j < m; ++j) {
                    const Acc a = s_a[j * (j + 1) / 2 + i];
#pragma unroll
                    for (int k = 0; k < NR; ++k) y[k] += a * (Acc)s_w[j * NR + k];
                }
            } else {
                for (int j = 0; j < m; ++j) {
                    const T a = s_a[j <= i ? ri + j : j * (j + 1) / 2 + i];
#pragma unroll
                    for (int k = 0; k < NR; ++k) y[k] += a * s_x[j * NR + k];
                }
            }
            if (d >= 0) {                        // < 0: masked entry
                T* dst = x + (int64_t)d * NR;
#pragma unroll
                for (int k = 0; k < NR; ++k) dst[k] = xo[k] + y[k];
            }
        }
    }
}

// Transfers for aggregates with |omega| <= SMALL_M, one thread per coarse DOF for
// the restriction and per aggregate entry for the prolongation, each for all NR
// right-hand sides (the index and the Z entry are loaded once for the NR products;
// AL: the NR interleaved values of a DOF are 16-byte aligned and load as 16-byte
// vectors); four independent entries (modes) per step, summed in four partial sums
// added in a fixed order.
template <typename T, int NR, bool AL>
__device__ inline void load_nr(const T* p, T (&v)[NR]) {
    const T* q = AL ? static_cast<const T*>(__builtin_assume_aligned(p, 16)) : p;
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = q[k];
}

template <typename T, int NR, bool AL>
__global__ void __launch_bounds__(WG) k_restrict_small(int64_t nc, const int32_t* agg_of_c, const int64_t* agg_ptr,
                                                       const int32_t* agg_dofs, const int64_t* zoff,
                                                       const int64_t* coff, const T* Zc, const T* t, T* rc) {
    for (int64_t c = blockIdx.x * (int64_t)WG + tid(); c < nc; c += (int64_t)gridDim.x * WG) {
        const int ag = agg_of_c[c];
        if (ag < 0) continue;
        const int64_t a0 = agg_ptr[ag];
        const int nw = (int)(agg_ptr[ag + 1] - a0);
        const T* z = Zc + zoff[ag] + (c - coff[ag]) * nw;
        const int32_t* dd = agg_dofs + a0;
        // four independent entries per step: their indices, then their gathers
        T acc[4][NR];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[u][k] = 0;
        int a = 0;
        for (; a + 4 <= nw; a += 4) {
            int32_t d[4];
            T zz[4], tv[4][NR];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                d[u] = dd[a + u];
                zz[u] = z[a + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) load_nr<T, NR, AL>(t + (int64_t)d[u] * NR, tv[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < NR; ++k) acc[u][k] += zz[u] * tv[u][k];
        }
        for (; a < nw; ++a) {
            T tv[NR];
            const T zz = z[a];
            load_nr<T, NR, AL>(t + (int64_t)dd[a] * NR, tv);
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[0][k] += zz * tv[k];
        }
        T* out = AL ? static_cast<T*>(__builtin_assume_aligned(rc + c * NR, 16)) : rc + c * NR;
#pragma unroll
        for (int k = 0; k < NR; ++k) out[k] = (acc[0][k] + acc[1][k]) + (acc[2][k] + acc[3][k]);
    }
}

template <typename T, int NR, bool AL>
__global__ void __launch_bounds__(WG) k_prolong_small(int64_t na, const int32_t* agg_of_p, const int64_t* agg_ptr,
                                                      const int32_t* agg_dofs, const int64_t* zoff,
                                                      const int32_t* k, const int64_t* coff, const T* Zc,
                                                      const T* ec, T* x) {
    for (int64_t p = blockIdx.x * (int64_t)WG + tid(); p < na; p += (int64_t)gridDim.x * WG) {
        const int ag = agg_of_p[p];
        if (ag < 0) continue;
        const int64_t a0 = agg_ptr[ag];
        const int nw = (int)(agg_ptr[ag + 1] - a0);
        const int kk = k[ag];
        const T* z = Zc + zoff[ag] + (p - a0);
        const T* ev = ec + coff[ag] * NR;
        T acc[4][NR];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[u][q] = 0;
        int s = 0;
        for (; s + 4 <= kk; s += 4) {
            T zz[4], e[4][NR];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                zz[u] = z[(int64_t)(s + u) * nw];
                load_nr<T, NR, AL>(ev + (int64_t)(s + u) * NR, e[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q) acc[u][q] += zz[u] * e[u][q];
        }
        for (; s < kk; ++s) {
            T e[NR];
            const T zz = z[(int64_t)s * nw];
            load_nr<T, NR, AL>(ev + (int64_t)s * NR, e);
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[0][q] += zz * e[q];
        }
        T* dst = x + (int64_t)agg_dofs[p] * NR;
        if (AL) dst = static_cast<T*>(__builtin_assume_aligned(dst, 16));
        T old[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) old[q] = dst[q];
#pragma unroll
        for (int q = 0; q < NR; ++q) dst[q] = old[q] + ((acc[0][q] + acc[1][q]) + (acc[2][q] + acc[3][q]));
    }
}

__global__ void k_gather_rhs(int64_t n, int nr, const double* b, int64_t ldb, double* B) {
    for (int64_t e = blockIdx.x * (int64_t)WG + tid(); e < n * NB; e += (int64_t)gridDim.x * WG) {
        const int64_t d = e / NB;
        const int k = (int)(e % NB);
        B[e] = k < nr ? b[k * ldb + d] : 0.0;
    }
}

__global__ void k_scatter_sol(int64_t n, int nr, const double* X, double* x, int64_t ldx) {
    for (int64_t e = blockIdx.x * (int64_t)WG + tid(); e < n * NB; e += (int64_t)gridDim.x * WG) {
        const int64_t d = e / NB;
        const int k = (int)(e % NB);
        if (k < nr) x[k * ldx + d] = X[e];
    }
}

// ---------------------------------------------------------------- segmented PCG
// Block b of the table covers DOFs [lo, hi) of one segment; thread = (DOF lane,
// right-hand side), a fixed-order tree over the DOF lanes gives NR sums.
template <int NR>
__global__ void __launch_bounds__(WG) k_seg_dot(const int64_t* blk_lo, const int64_t* blk_hi, const double* a0,
                                                const double* b0, const double* a1, const double* b1, double* part,
                                                int n_blk) {
    __shared__ double s_r[2][WG];
    const int b = blockIdx.x;
    const int k = tid() % NR, dl = tid() / NR;
    constexpr int DL = WG / NR;
    double u = 0.0, v = 0.0;
    for (int64_t d = blk_lo[b] + dl; d < blk_hi[b]; d += DL) {
        const int64_t e = d * NR + k;
        u += a0[e] * b0[e];
        if (a1) v += a1[e] * b1[e];
    }
    s_r[0][tid()] = u;
    s_r[1][tid()] = v;
    __syncthreads();
    for (int off = WG / 2; off >= NR; off >>= 1) {
        if (tid() < off) {
            s_r[0][tid()] += s_r[0][tid() + off];
            s_r[1][tid()] += s_r[1][tid() + off];
        }
        __syncthreads();
    }
    if (tid() < NR) {
        part[(int64_t)b * NR + tid()] = s_r[0][tid()];
        part[((int64_t)n_blk + b) * NR + tid()] = s_r[1][tid()];
    }
}

// out[s * NR + k] = sum over the blocks of segment s, in block order
// One wave per (segment, right-hand side): lane l sums the blocks l, l + 64, ... of
// the segment in order, then a butterfly over the lanes -- a fixed order, so the
// same partials always give the same sum.
__global__ void k_seg_sum(int n_seg, int nr, const int32_t* seg_blk, const double* part, int n_blk, double* out0,
                          double* out1) {
    const int i = (int)((blockIdx.x * WG + tid()) >> 6), lane = tid() & 63;
    if (i >= n_seg * nr) return;
    const int s = i / nr, k = i % nr;
    double u = 0.0, v = 0.0;
    for (int b = seg_blk[s] + lane; b < seg_blk[s + 1]; b += 64) {
        u += part[(int64_t)b * nr + k];
        v += part[((int64_t)n_blk + b) * nr + k];
    }
    for (int off = 32; off > 0; off >>= 1) {
        u += __shfl_xor(u, off, 64);
        v += __shfl_xor(v, off, 64);
    }
    if (lane == 0) {
        out0[i] = u;
        if (out1) out1[i] = v;
    }
}

__global__ void k_pcg_init(int n_s, const double* bb, int32_t* act, int32_t* iters, double* relres,
                           int32_t* it_flag) {
    const int i = blockIdx.x * WG + tid();
    if (i == 0) {
        it_flag[0] = 0;
        it_flag[1] = 0;
    }
    if (i >= n_s) return;
    act[i] = bb[i] > 0.0 ? 1 : 0;
    iters[i] = 0;
    relres[i] = bb[i] > 0.0 ? 1.0 : 0.0;
}

__global__ void k_pcg_alpha(int n_s, const int32_t* act, const double* rz, const double* pq, double* alpha,
                            int32_t* flag) {
    const int i = blockIdx.x * WG + tid();
    if (i >= n_s) return;
    double a = 0.0;
    if (act[i]) {
        const double d = pq[i];
        // breakdown cause bits: 1 p^T A p <= 0, 2 p^T A p or r^T z not finite
        if (!isfinite(d) || !isfinite(rz[i])) atomicOr(flag, 2);
        else if (!(d > 0.0)) atomicOr(flag, 1);
        else a = rz[i] / d;
    }
    alpha[i] = a;
}

template <int NR>
__global__ void __launch_bounds__(WG) k_pcg_update_xr(const int32_t* blk_seg, const int64_t* blk_lo,
                                                      const int64_t* blk_hi, const int32_t* act, const double* alpha,
                                                      const double* p, const double* q, double* x, double* r,
                                                      double* part) {
    __shared__ double s_r[WG];
    const int b = blockIdx.x;
    const int k = tid() % NR, dl = tid() / NR;
    constexpr int DL = WG / NR;
    const int i = blk_seg[b] * NR + k;
    const bool on = act[i] != 0;
    const double a = alpha[i];
    double u = 0.0;
    for (int64_t d = blk_lo[b] + dl; d < blk_hi[b]; d += DL) {
        const int64_t e = d * NR + k;
        double re = r[e];
        if (on) {
            x[e] += a * p[e];
            re -= a * q[e];
            r[e] = re;
        }
        u += re * re;
    }
    s_r[tid()] = u;
    __syncthreads();
    for (int off = WG / 2; off >= NR; off >>= 1) {
        if (tid() < off) s_r[tid()] += s_r[tid() + off];
        __syncthreads();
    }
    if (tid() < NR) part[(int64_t)b * NR + tid()] = s_r[tid()];
}

// single workgroup: state transitions and the active count (fixed-order sum)
__global__ void __launch_bounds__(WG) k_pcg_check(int n_s, int32_t* it_dev, double tol2, const double* bb,
                                                  const double* rr, int32_t* act, int32_t* iters, double* relres,
                                                  int32_t* count, int32_t* flag) {
    __shared__ int s_c[WG];
    const int it = it_dev[0] + 1;
    int c = 0;
    for (int i = tid(); i < n_s; i += WG) {
        if (!act[i]) continue;
        const double v = rr[i];
        if (!isfinite(v)) {
            atomicOr(flag, 4);          // residual norm not finite
            continue;
        }
        relres[i] = sqrt(v / bb[i]);
        iters[i] = it;
        if (v <= tol2 * bb[i]) act[i] = 0;
        else ++c;
    }
    s_c[tid()] = c;
    __syncthreads();
    for (int off = WG / 2; off > 0; off >>= 1) {
        if (tid() < off) s_c[tid()] += s_c[tid() + off];
        __syncthreads();
    }
    if (tid() == 0) {
        count[0] = s_c[0];
        it_dev[0] = it;
    }
}

__global__ void k_pcg_beta(int n_s, const int32_t* act, const double* rz_new, const double* rz_old_dot, double* rz,
                           double* beta, int32_t* flag) {
    const int i = blockIdx.x * WG + tid();
    if (i >= n_s) return;
    double bt = 0.0;
    if (act[i]) {
        const double num = rz_old_dot ? rz_new[i] - rz_old_dot[i] : rz_new[i];
        bt = num / rz[i];
        if (!isfinite(bt)) atomicOr(flag, 8);   // beta not finite
        rz[i] = rz_new[i];
    }
    beta[i] = bt;
}

template <int NR>
__global__ void __launch_bounds__(WG) k_pcg_update_p(const int32_t* blk_seg, const int64_t* blk_lo,
                                                     const int64_t* blk_hi, const int32_t* act, const double* beta,
                                                     const double* z, double* p) {
    const int b = blockIdx.x;
    const int k = tid() % NR, dl = tid() / NR;
    constexpr int DL = WG / NR;
    const int i = blk_seg[b] * NR + k;
    if (!act[i]) return;
    const double bt = beta[i];
    for (int64_t d = blk_lo[b] + dl; d < blk_hi[b]; d += DL) {
        const int64_t e = d * NR + k;
        p[e] = z[e] + bt * p[e];
    }
}

__global__ void k_pcg_start(int64_t len, const double* b, double* r, double* x) {
    for (int64_t e = blockIdx.x * (int64_t)WG + tid(); e < len; e += (int64_t)gridDim.x * WG) {
        r[e] = b[e];
        x[e] = 0.0;
    }
}

}  // namespace

// ====================================================================== launchers

// The residual rows of a supernode-blocked level by supernode row blocks, for blocks
// of NB right-hand sides: L lanes per block (blk as in k_sup_resid_blocks) take its
// shared column list; per entry a lane gathers the NB interleaved x values once and
// uses them for up to 4 rows of the block at a time (slots past the block's end
// repeat its last row and are never stored).  Per row the products, the per-lane
// sums and the cross-lane sums are those of k_csr_resid_rows_s for the same L: the
// results are bit-identical to it.
template <typename T, int L>
__global__ void __launch_bounds__(WG) k_sup_resid_blocks_s(int64_t nblk, const int32_t* blk, const int32_t* rows,
                                                           const int64_t* rowptr, const int32_t* scol,
                                                           const int64_t* scoff, const T* val, const T* x,
                                                           const T* r, T* out, int x_zero) {
    constexpr int RB = 4;
    const int lane = tid() & (L - 1);
    const int64_t stride = (int64_t)gridDim.x * (WG / L);
    for (int64_t b = ((int64_t)blockIdx.x * WG + tid()) / L; b < nblk; b += stride) {
        const int32_t t0 = blk[2 * b], nb = blk[2 * b + 1];
        const int32_t p0 = rows[t0];
        const int64_t q0 = rowptr[p0], q1 = rowptr[p0 + 1];
        const int64_t cb = scoff[p0] - q0;   // the list entry of position q is scol[cb + q]
        for (int j0 = 0; j0 < nb; j0 += RB) {
            int32_t p[RB];
            int64_t vo[RB];   // value offset of row j relative to the first row's
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                p[j] = rows[t0 + min(j0 + j, nb - 1)];
                vo[j] = rowptr[p[j]] - q0;
            }
            T s[RB][NB];
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
                for (int k = 0; k < NB; ++k) s[j][k] = 0;
            if (!x_zero) {
                const int nit = (int)((q1 - q0 + L - 1) / L);
                for (int it = 0; it < nit; it += 2) {
                    const int64_t qa = q0 + lane + (int64_t)it * L, qb = qa + L;
                    const int64_t qac = qa < q1 ? qa : q1 - 1, qbc = qb < q1 ? qb : q1 - 1;
                    const int32_t ca = scol[cb + qac], cc = scol[cb + qbc];
                    T va[RB], vb[RB];
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        va[j] = val[vo[j] + qac];
                        vb[j] = val[vo[j] + qbc];
                    }
                    T xa[NB], xb[NB];
                    load_xrow(x + (int64_t)ca * NB, xa);
                    load_xrow(x + (int64_t)cc * NB, xb);
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        const T wa = qa < q1 ? va[j] : (T)0, wb = qb < q1 ? vb[j] : (T)0;
#pragma unroll
                        for (int k = 0; k < NB; ++k) s[j][k] += wa * xa[k];
#pragma unroll
                        for (int k = 0; k < NB; ++k) s[j][k] += wb * xb[k];
                    }
                }
            }
            constexpr int PL = L < NB ? NB / L : 1;   // right-hand sides per writing lane
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                slot_reduce<T, L>(s[j], lane);
                if (j0 + j < nb && lane * PL < NB)
#pragma unroll
                    for (int i = 0; i < PL; ++i) {
                        const int k = lane * PL + i;
                        out[(int64_t)(t0 + j0 + j) * NB + k] = r[(int64_t)p[j] * NB + k] - s[j][i];
                    }
            }
        }
    }
}

template <typename T>
void launch_sup_resid_blocks_b(int64_t nblk, const int32_t* blk, const int32_t* rows, const int64_t* rowptr,
                               const int32_t* scol, const int64_t* scoff, const T* val, const T* x, const T* r, T* out,
                               bool x_zero, int lanes, hipStream_t st) {
    if (nblk <= 0) return;
    const int xz = x_zero ? 1 : 0;
    if (lanes <= 4)
        hipLaunchKernelGGL((k_sup_resid_blocks_s<T, 4>), dim3(grid_for(nblk * 4)), dim3(WG), 0, st, nblk, blk, rows,
                           rowptr, scol, scoff, val, x, r, out, xz);
    else if (lanes <= 8)
        hipLaunchKernelGGL((k_sup_resid_blocks_s<T, 8>), dim3(grid_for(nblk * 8)), dim3(WG), 0, st, nblk, blk, rows,
                           rowptr, scol, scoff, val, x, r, out, xz);
    else
        hipLaunchKernelGGL((k_sup_resid_blocks_s<T, 16>), dim3(grid_for(nblk * 16)), dim3(WG), 0, st, nblk, blk,
                           rows, rowptr, scol, scoff, val, x, r, out, xz);
}

template <typename T>
void launch_csr_resid_rows_b(int64_t nrows, const int32_t* rows, const int64_t* rowptr, const int32_t* col,
                             const T* val, const T* x, const T* r, T* out, bool x_zero, int lanes, hipStream_t st,
                             const int64_t* scoff) {
    if (nrows <= 0) return;
    if (lanes <= 4)
        hipLaunchKernelGGL((k_csr_resid_rows_s<T, 4>), dim3(grid_for(nrows * 4)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, x_zero ? 1 : 0, scoff);
    else if (lanes <= 8)
        hipLaunchKernelGGL((k_csr_resid_rows_s<T, 8>), dim3(grid_for(nrows * 8)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, x_zero ? 1 : 0, scoff);
    else if (lanes <= 16)
        hipLaunchKernelGGL((k_csr_resid_rows_s<T, 16>), dim3(grid_for(nrows * 16)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, x_zero ? 1 : 0, scoff);
    else if (lanes >= 64)
        hipLaunchKernelGGL((k_csr_resid_rows_b<T, 64>), dim3(grid_for(nrows * 64)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, x_zero ? 1 : 0, scoff);
    else
        hipLaunchKernelGGL((k_csr_resid_rows_b<T, 32>), dim3(grid_for(nrows * 32)), dim3(WG), 0, st, nrows, rows,
                           rowptr, col, val, x, r, out, x_zero ? 1 : 0, scoff);
}

template <typename T>
void launch_csr_spmv_b(int64_t n, const int64_t* rowptr, const int32_t* col, const T* val, const T* x, T* y,
                       const T* r_minus, int lanes, hipStream_t st, const int64_t* scoff) {
    if (n <= 0) return;
    if (lanes <= 4)
        hipLaunchKernelGGL((k_csr_spmv_s<T, 4>), dim3(grid_for(n * 4)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else if (lanes <= 8)
        hipLaunchKernelGGL((k_csr_spmv_s<T, 8>), dim3(grid_for(n * 8)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else if (lanes <= 16)
        hipLaunchKernelGGL((k_csr_spmv_s<T, 16>), dim3(grid_for(n * 16)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else if (lanes >= 64)
        hipLaunchKernelGGL((k_csr_spmv_b<T, 64>), dim3(grid_for(n * 64)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
    else
        hipLaunchKernelGGL((k_csr_spmv_b<T, 32>), dim3(grid_for(n * 32)), dim3(WG), 0, st, n, rowptr, col, val, x, y,
                           r_minus, scoff);
}

template <typename T>
void launch_sub_symv_b(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                       const T* tiles, const T* rloc, const int64_t* scr_off, T* scr, int chl, hipStream_t st) {
    if (n_items <= 0) return;
    hipEvent_t e0, e1;
    if (take_launch_events(&e0, &e1))
        hipExtLaunchKernelGGL(k_sub_symv_b<T>, dim3((unsigned)n_items), dim3(WG), 0, st, e0, e1, 0, items, sub_off,
                              tp_off, tiles, rloc, scr_off, scr, chl);
    else
        hipLaunchKernelGGL(k_sub_symv_b<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, sub_off, tp_off, tiles,
                           rloc, scr_off, scr, chl);
}

template <typename T>
void launch_sub_finalize_b(int64_t r0, int64_t r1, const int32_t* pos_sub, const int64_t* sub_off,
                           const int64_t* scr_off, const T* scr, const int32_t* sub_dofs, T* x, bool accumulate,
                           int chl, int fl, hipStream_t st) {
    if (r1 <= r0) return;
    if (fl >= 32)
        hipLaunchKernelGGL((k_sub_finalize_b<T, 32>), dim3(grid_for(r1 - r0, WG / 32)), dim3(WG), 0, st, r0, r1,
                           pos_sub, sub_off, scr_off, scr, sub_dofs, x, accumulate ? 1 : 0, chl);
    else
        hipLaunchKernelGGL((k_sub_finalize_b<T, 8>), dim3(grid_for(r1 - r0, WG / 8)), dim3(WG), 0, st, r0, r1,
                           pos_sub, sub_off, scr_off, scr, sub_dofs, x, accumulate ? 1 : 0, chl);
}

// The same sums from the per-entry address table of the single-vector finalize
// (int4 per overlap entry: row-part address, column-part address + J * 64 + l, J,
// row-part chunks | tile rows << 16, in single-vector units; the block layout holds
// NB consecutive values at NB times that address): one table load replaces the
// entry's subdomain and offset lookups.  Same per-thread subsets, same order, same
// results as k_sub_finalize_b with accumulate.
template <typename T, int FL>
__global__ void __launch_bounds__(WG) k_sub_finalize_tab_b(int64_t r0, int64_t r1, const int4* tab, const T* scr,
                                                           const int32_t* sub_dofs, T* x) {
    constexpr int ND = WG / FL;
    __shared__ T s_y[FL][ND][NB];
    const int dl = tid() % ND, j = tid() / ND;
    const int64_t t = r0 + (int64_t)blockIdx.x * ND + dl;
    T y[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) y[q] = 0;
    if (t < r1) {
        const int4 e = tab[t];
        const T* part = scr + (int64_t)(uint32_t)e.x * NB;
        const T* colpart = scr + (int64_t)(uint32_t)e.y * NB;
        const int J = e.z, nch = e.w & 0xffff, nt = e.w >> 16;
        const int K = nch + (nt - 1 - J);
        for (int k = j; k < K; k += FL) {
            const int64_t I = J + 1 + (k - nch);
            const T* src = k < nch ? part + (int64_t)k * 64 * NB : colpart + I * (I - 1) / 2 * 64 * NB;
#pragma unroll
            for (int q = 0; q < NB; ++q) y[q] += src[q];
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) s_y[j][dl][q] = y[q];
    __syncthreads();
    if (j < NB && t < r1) {
        T v = s_y[0][dl][j];
        for (int q = 1; q < FL; ++q) v += s_y[q][dl][j];
        const int64_t d = sub_dofs[t];   // < 0: masked entry
        if (d >= 0) x[d * NB + j] = x[d * NB + j] + v;
    }
}

template <typename T>
void launch_sub_finalize_tab_b(int64_t r0, int64_t r1, const int32_t* tab, const T* scr, const int32_t* sub_dofs,
                               T* x, int fl, hipStream_t st) {
    if (r1 <= r0) return;
    const int4* tb = reinterpret_cast<const int4*>(tab);
    if (fl >= 32)
        hipLaunchKernelGGL((k_sub_finalize_tab_b<T, 32>), dim3(grid_for(r1 - r0, WG / 32)), dim3(WG), 0, st, r0, r1,
                           tb, scr, sub_dofs, x);
    else
        hipLaunchKernelGGL((k_sub_finalize_tab_b<T, 8>), dim3(grid_for(r1 - r0, WG / 8)), dim3(WG), 0, st, r0, r1,
                           tb, scr, sub_dofs, x);
}

template <typename T>
void launch_restrict_b(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                       const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* t, T* rc,
                       hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_restrict_b<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, agg_ptr, agg_dofs, zoff, k,
                       coff, Zc, t, rc);
}

template <typename T>
void launch_prolong_b(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                      const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                      hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_prolong_b<T>, dim3((unsigned)n_items), dim3(WG), 0, st, items, agg_ptr, agg_dofs, zoff, k,
                       coff, Zc, ec, x);
}

void launch_gather_rhs(int64_t n, int32_t nr, const double* b, int64_t ldb, double* B, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rhs, dim3(grid_for(n * NB)), dim3(WG), 0, st, n, (int)nr, b, ldb, B);
}

void launch_scatter_sol(int64_t n, int32_t nr, const double* X, double* x, int64_t ldx, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_sol, dim3(grid_for(n * NB)), dim3(WG), 0, st, n, (int)nr, X, x, ldx);
}

void launch_seg_dot(const SegTable& t, int nr, const double* a0, const double* b0, const double* a1,
                    const double* b1, double* part, double* out0, double* out1, hipStream_t st) {
    if (nr == NB)
        hipLaunchKernelGGL(k_seg_dot<NB>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_lo, t.blk_hi, a0, b0, a1,
                           b1, part, t.n_blk);
    else
        hipLaunchKernelGGL(k_seg_dot<1>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_lo, t.blk_hi, a0, b0, a1, b1,
                           part, t.n_blk);
    hipLaunchKernelGGL(k_seg_sum, dim3(grid_for((int64_t)t.n_seg * nr * 64)), dim3(WG), 0, st, t.n_seg, nr, t.seg_blk,
                       part, t.n_blk, out0, a1 ? out1 : nullptr);
}

void launch_pcg_init(int n_s, const double* bb, int32_t* act, int32_t* iters, double* relres, int32_t* it_flag,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_init, dim3(grid_for(n_s)), dim3(WG), 0, st, n_s, bb, act, iters, relres, it_flag);
}

void launch_pcg_alpha(int n_s, const int32_t* act, const double* rz, const double* pq, double* alpha, int32_t* flag,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_alpha, dim3(grid_for(n_s)), dim3(WG), 0, st, n_s, act, rz, pq, alpha, flag);
}

void launch_pcg_update_xr(const SegTable& t, int nr, const int32_t* act, const double* alpha, const double* p,
                          const double* q, double* x, double* r, double* part, double* rr, hipStream_t st) {
    if (nr == NB)
        hipLaunchKernelGGL(k_pcg_update_xr<NB>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_seg, t.blk_lo,
                           t.blk_hi, act, alpha, p, q, x, r, part);
    else
        hipLaunchKernelGGL(k_pcg_update_xr<1>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_seg, t.blk_lo,
                           t.blk_hi, act, alpha, p, q, x, r, part);
    hipLaunchKernelGGL(k_seg_sum, dim3(grid_for((int64_t)t.n_seg * nr * 64)), dim3(WG), 0, st, t.n_seg, nr, t.seg_blk,
                       part, 0, rr, nullptr);
}

void launch_pcg_check(int n_s, int32_t* it_dev, double tol2, const double* bb, const double* rr, int32_t* act,
                      int32_t* iters, double* relres, int32_t* count, int32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(WG), 0, st, n_s, it_dev, tol2, bb, rr, act, iters, relres, count,
                       flag);
}

void launch_pcg_beta(int n_s, const int32_t* act, const double* rz_new, const double* rz_old_dot, double* rz,
                     double* beta, int32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_beta, dim3(grid_for(n_s)), dim3(WG), 0, st, n_s, act, rz_new, rz_old_dot, rz, beta,
                       flag);
}

void launch_pcg_update_p(const SegTable& t, int nr, const int32_t* act, const double* beta, const double* z,
                         double* p, hipStream_t st) {
    if (nr == NB)
        hipLaunchKernelGGL(k_pcg_update_p<NB>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_seg, t.blk_lo,
                           t.blk_hi, act, beta, z, p);
    else
        hipLaunchKernelGGL(k_pcg_update_p<1>, dim3((unsigned)t.n_blk), dim3(WG), 0, st, t.blk_seg, t.blk_lo,
                           t.blk_hi, act, beta, z, p);
}

void launch_pcg_start(int64_t len, const double* b, double* r, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_start, dim3(grid_for(len)), dim3(WG), 0, st, len, b, r, x);
}

template <typename T, int NR>
void launch_small_sub(int64_t s0, int64_t n_sub, const int64_t* sub_off, const int32_t* sub_dofs,
                      const int64_t* pk_off, const T* pk, const T* rloc, T* x, int max_m, hipStream_t st,
                      bool fact) {
    if (n_sub <= 0) return;
    if (max_m < 1 || max_m > SMALL_M) throw std::runtime_error("launch_small_sub: max_m outside 1 .. SMALL_M");
    if (n_sub > INT32_MAX) throw std::runtime_error("launch_small_sub: more than 2^31 - 1 subdomains");
    const size_t lds = ((size_t)max_m * (max_m + 1) / 2 + (fact ? 2 : 1) * (size_t)max_m * NR) * sizeof(T);
    // persistent waves: as many as fit on the device at once (LDS or registers bound)
    auto kern = fact ? &k_small_sub<T, NR, true> : &k_small_sub<T, NR, false>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), 64, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (size_t)(160 * 1024) / lds));
    const unsigned grid = (unsigned)std::min<int64_t>(n_sub, (int64_t)per_cu * device_cu_count());
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, st, (int32_t)s0, (int32_t)n_sub, sub_off, sub_dofs, pk_off,
                       pk, rloc, x, max_m);
}

template <typename T, int NR>
void launch_restrict_small(int64_t nc, const int32_t* agg_of_c, const int64_t* agg_ptr, const int32_t* agg_dofs,
                           const int64_t* zoff, const int64_t* coff, const T* Zc, const T* t, T* rc, hipStream_t st) {
    if (nc <= 0) return;
    if ((NR * sizeof(T)) % 16 == 0 && (((uintptr_t)t | (uintptr_t)rc) & 15) == 0)
        hipLaunchKernelGGL((k_restrict_small<T, NR, true>), dim3(grid_for(nc)), dim3(WG), 0, st, nc, agg_of_c,
                           agg_ptr, agg_dofs, zoff, coff, Zc, t, rc);
    else
        hipLaunchKernelGGL((k_restrict_small<T, NR, false>), dim3(grid_for(nc)), dim3(WG), 0, st, nc, agg_of_c,
                           agg_ptr, agg_dofs, zoff, coff, Zc, t, rc);
}

template <typename T, int NR>
void launch_prolong_small(int64_t na, const int32_t* agg_of_p, const int64_t* agg_ptr, const int32_t* agg_dofs,
                          const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                          hipStream_t st) {
    if (na <= 0) return;
    if ((NR * sizeof(T)) % 16 == 0 && (((uintptr_t)ec | (uintptr_t)x) & 15) == 0)
        hipLaunchKernelGGL((k_prolong_small<T, NR, true>), dim3(grid_for(na)), dim3(WG), 0, st, na, agg_of_p,
                           agg_ptr, agg_dofs, zoff, k, coff, Zc, ec, x);
    else
        hipLaunchKernelGGL((k_prolong_small<T, NR, false>), dim3(grid_for(na)), dim3(WG), 0, st, na, agg_of_p,
                           agg_ptr, agg_dofs, zoff, k, coff, Zc, ec, x);
}

#define LSDD_SMALL_INST(T, NR)                                                                                     \
    template void launch_small_sub<T, NR>(int64_t, int64_t, const int64_t*, const int32_t*, const int64_t*,        \
                                          const T*, const T*, T*, int, hipStream_t, bool);                          \
    template void launch_restrict_small<T, NR>(int64_t, const int32_t*, const int64_t*, const int32_t*,            \
                                               const int64_t*, const int64_t*, const T*, const T*, T*, hipStream_t); \
    template void launch_prolong_small<T, NR>(int64_t, const int32_t*, const int64_t*, const int32_t*,             \
                                              const int64_t*, const int32_t*, const int64_t*, const T*, const T*,   \
                                              T*, hipStream_t);
LSDD_SMALL_INST(double, 1)
LSDD_SMALL_INST(double, NRB)
LSDD_SMALL_INST(float, 1)
LSDD_SMALL_INST(float, NRB)

#define LSDD_BLK_INST(T)                                                                                            \
    template void launch_sup_resid_blocks_b<T>(int64_t, const int32_t*, const int32_t*, const int64_t*,            \
                                               const int32_t*, const int64_t*, const T*, const T*, const T*, T*,     \
                                               bool, int, hipStream_t);                                              \
    template void launch_csr_resid_rows_b<T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const T*,      \
                                             const T*, const T*, T*, bool, int, hipStream_t, const int64_t*);         \
    template void launch_csr_spmv_b<T>(int64_t, const int64_t*, const int32_t*, const T*, const T*, T*, const T*,    \
                                       int, hipStream_t, const int64_t*);                                             \
    template void launch_sub_symv_b<T>(int64_t, const int32_t*, const int64_t*, const int64_t*, const T*, const T*,  \
                                       const int64_t*, T*, int, hipStream_t);                                         \
    template void launch_sub_finalize_tab_b<T>(int64_t, int64_t, const int32_t*, const T*, const int32_t*, T*, int, \
                                               hipStream_t);                                                          \
    template void launch_sub_finalize_b<T>(int64_t, int64_t, const int32_t*, const int64_t*, const int64_t*,         \
                                           const T*, const int32_t*, T*, bool, int, int, hipStream_t);                \
    template void launch_restrict_b<T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const int64_t*,      \
                                       const int32_t*, const int64_t*, const T*, const T*, T*, hipStream_t);          \
    template void launch_prolong_b<T>(int64_t, const int32_t*, const int64_t*, const int32_t*, const int64_t*,       \
                                      const int32_t*, const int64_t*, const T*, const T*, T*, hipStream_t);
LSDD_BLK_INST(double)
LSDD_BLK_INST(float)

}  // namespace lsdd
