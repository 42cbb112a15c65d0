// FP64 matrix-core tile contraction for gfx950 (v_mfma_f64_16x16x4f64), and an
// FP32 variant (v_mfma_f32_16x16x4f32) at the end.
//
// One workgroup of 256 threads (4 waves) accumulates a 64 x 64 output tile
//     acc[i][j] = sum_k a(k, i) * b(k, j),   i in [m0, m0+64), j in [n0, n0+64)
// over k in [kbeg, kend).  K is staged through LDS in chunks of 32 (register
// prefetch of the next chunk while the matrix cores work on the current one).
// Each wave owns a 32 x 32 quarter as 2 x 2 blocks of 16 x 16.
//
// Operand layouts (element (k, i) of a K x M operand with leading dimension ld):
//   KMAJ: p[k + i * ld]   (k contiguous; e.g. A of A^T B, column-major)
//   IMAJ: p[i + k * ld]   (i contiguous; e.g. a column block L[:, k0:k1])
// Out-of-range elements (i >= ilim or k >= kend) are read as zero.
//
// Lane layout of the 16x16x4 FP64 instruction (checked on gfx950): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result register v of lane
// l holds D[l / 16 + 4 v][l % 16].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsdd {
namespace mg {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int T = 64;        // output tile edge
constexpr int KC = 32;       // K chunk per LDS stage
constexpr int LS = KC + 2;   // LDS row stride in doubles (conflict-free fragment reads)
constexpr int NT = 256;

enum { KMAJ = 0, IMAJ = 1 };

struct Smem {
    double a[T][LS];
    double b[T][LS];
};

// Each thread fetches 8 elements of the 64 x 32 chunk; the mapping keeps
// global reads contiguous along the operand's fast index.
template <int LAY>
__device__ inline void chunk_idx(int q, int& i, int& k) {
    const int t = (int)threadIdx.x;
    if (LAY == KMAJ) {
        k = t & 31;
        i = (t >> 5) + 8 * q;
    } else {
        i = t & 63;
        k = (t >> 6) + 4 * q;
    }
}

template <int LAY>
__device__ inline void fetch(const double* __restrict__ p, int64_t ld, int i0, int ilim, int k0, int kend,
                             double (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int i, k;
        chunk_idx<LAY>(q, i, k);
        const int gi = i0 + i, gk = k0 + k;
        double v = 0.0;
        if (gi < ilim && gk < kend)
            v = (LAY == KMAJ) ? p[gk + (int64_t)gi * ld] : p[gi + (int64_t)gk * ld];
        r[q] = v;
    }
}

template <int LAY>
__device__ inline void stash(double (*s)[LS], const double (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int i, k;
        chunk_idx<LAY>(q, i, k);
        s[i][k] = r[q];
    }
}

__device__ inline void zero(d4 (&acc)[2][2]) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
}

// acc += sum over k in [kbeg, kend) of a(k, m0 + .) b(k, n0 + .); a has ilim = M
// valid rows, b has N valid columns.  Must be called by all 256 threads.
template <int LA, int LB>
__device__ inline void tile_mma(Smem& sm, const double* __restrict__ a, int64_t lda, int m0, int M,
                                const double* __restrict__ b, int64_t ldb, int n0, int N, int kbeg, int kend,
                                d4 (&acc)[2][2]) {
    if (kbeg >= kend) return;
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int lm = l & 15, lk = l >> 4;
    double ra[8], rb[8];
    fetch<LA>(a, lda, m0, M, kbeg, kend, ra);
    fetch<LB>(b, ldb, n0, N, kbeg, kend, rb);
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
        __syncthreads();
        stash<LA>(sm.a, ra);
        stash<LB>(sm.b, rb);
        __syncthreads();
        if (k0 + KC < kend) {
            fetch<LA>(a, lda, m0, M, k0 + KC, kend, ra);
            fetch<LB>(b, ldb, n0, N, k0 + KC, kend, rb);
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const double a0 = sm.a[wr + lm][kk + lk], a1 = sm.a[wr + 16 + lm][kk + lk];
            const double b0 = sm.b[wc + lm][kk + lk], b1 = sm.b[wc + 16 + lm][kk + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
}

// Tile coordinates (row, column inside the 64 x 64 tile) of accumulator
// register v of block (p, q) held by this thread.
__device__ inline int acc_row(int p, int v) {
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    return (w & 1) * 32 + 16 * p + (l >> 4) + 4 * v;
}
__device__ inline int acc_col(int q) {
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    return (w >> 1) * 32 + 16 * q + (l & 15);
}

// ---------------------------------------------------------------- FP32 variant
// The same 64 x 64 tile contraction on v_mfma_f32_16x16x4f32: the FP64
// operands are rounded to FP32 as they are staged in LDS and the products are
// accumulated in FP32.  The FP32 instruction takes its operands like the FP64
// one (lane l: A[l % 16][l / 16], B[l / 16][l % 16]) but returns register v of
// lane l as D[4 (l / 16) + v][l % 16] (acc_row32).

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LS32 = KC + 1;  // LDS row stride in floats

struct Smem32 {
    float a[T][LS32];
    float b[T][LS32];
};

template <int LAY>
__device__ inline void stash32(float (*s)[LS32], const double (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int i, k;
        chunk_idx<LAY>(q, i, k);
        s[i][k] = (float)r[q];
    }
}

__device__ inline void zero32(f4 (&acc)[2][2]) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
}

template <int LA, int LB>
__device__ inline void tile_mma32(Smem32& sm, const double* __restrict__ a, int64_t lda, int m0, int M,
                                  const double* __restrict__ b, int64_t ldb, int n0, int N, int kbeg, int kend,
                                  f4 (&acc)[2][2]) {
    if (kbeg >= kend) return;
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int lm = l & 15, lk = l >> 4;
    double ra[8], rb[8];
    fetch<LA>(a, lda, m0, M, kbeg, kend, ra);
    fetch<LB>(b, ldb, n0, N, kbeg, kend, rb);
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
        __syncthreads();
        stash32<LA>(sm.a, ra);
        stash32<LB>(sm.b, rb);
        __syncthreads();
        if (k0 + KC < kend) {
            fetch<LA>(a, lda, m0, M, k0 + KC, kend, ra);
            fetch<LB>(b, ldb, n0, N, k0 + KC, kend, rb);
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const float a0 = sm.a[wr + lm][kk + lk], a1 = sm.a[wr + 16 + lm][kk + lk];
            const float b0 = sm.b[wc + lm][kk + lk], b1 = sm.b[wc + 16 + lm][kk + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
}

__device__ inline int acc_row32(int p, int v) {
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    return (w & 1) * 32 + 16 * p + 4 * (l >> 4) + v;
}

// ---------------------------------------------------------------- 128 x 128 tiles
// The same contraction on a 128 x 128 output tile: each of the four waves owns a
// 64 x 64 quarter as 4 x 4 blocks of 16 x 16, so every operand entry staged in
// LDS feeds twice the products of the 64 x 64 tile and the operands cross the
// memory hierarchy half as often per product.  K is staged in chunks of 16.

constexpr int T2 = 128;
constexpr int KC2 = 16;
constexpr int LS2 = KC2 + 2;

struct Smem128 {
    double a[T2][LS2];
    double b[T2][LS2];
};

// 8 elements of the 128 x 16 chunk per thread, reads contiguous along the fast index
template <int LAY>
__device__ inline void chunk_idx2(int q, int& i, int& k) {
    const int t = (int)threadIdx.x;
    if (LAY == KMAJ) {
        k = t & 15;
        i = (t >> 4) + 16 * q;
    } else {
        i = t & 127;
        k = (t >> 7) + 2 * q;
    }
}

template <int LAY>
__device__ inline void fetch2(const double* __restrict__ p, int64_t ld, int i0, int ilim, int k0, int kend,
                              double (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int i, k;
        chunk_idx2<LAY>(q, i, k);
        const int gi = i0 + i, gk = k0 + k;
        double v = 0.0;
        if (gi < ilim && gk < kend) v = (LAY == KMAJ) ? p[gk + (int64_t)gi * ld] : p[gi + (int64_t)gk * ld];
        r[q] = v;
    }
}

template <int LAY>
__device__ inline void stash2(double (*s)[LS2], const double (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int i, k;
        chunk_idx2<LAY>(q, i, k);
        s[i][k] = r[q];
    }
}

__device__ inline void zero(d4 (&acc)[4][4]) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
}

// acc += sum over k in [kbeg, kend) of a(k, m0 + .) b(k, n0 + .) on a 128 x 128
// tile.  Must be called by all 256 threads.
template <int LA, int LB>
__device__ inline void tile_mma128(Smem128& sm, const double* __restrict__ a, int64_t lda, int m0, int M,
                                   const double* __restrict__ b, int64_t ldb, int n0, int N, int kbeg, int kend,
                                   d4 (&acc)[4][4]) {
    if (kbeg >= kend) return;
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const int wr = (w & 1) * 64, wc = (w >> 1) * 64;
    const int lm = l & 15, lk = l >> 4;
    double ra[8], rb[8];
    fetch2<LA>(a, lda, m0, M, kbeg, kend, ra);
    fetch2<LB>(b, ldb, n0, N, kbeg, kend, rb);
    for (int k0 = kbeg; k0 < kend; k0 += KC2) {
        __syncthreads();
        stash2<LA>(sm.a, ra);
        stash2<LB>(sm.b, rb);
        __syncthreads();
        if (k0 + KC2 < kend) {
            fetch2<LA>(a, lda, m0, M, k0 + KC2, kend, ra);
            fetch2<LB>(b, ldb, n0, N, k0 + KC2, kend, rb);
        }
#pragma unroll
        for (int kk = 0; kk < KC2; kk += 4) {
            double fa[4], fb[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) fa[p] = sm.a[wr + 16 * p + lm][kk + lk];
#pragma unroll
            for (int q = 0; q < 4; ++q) fb[q] = sm.b[wc + 16 * q + lm][kk + lk];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[p], fb[q], acc[p][q], 0, 0, 0);
        }
    }
}

// position inside the 128 x 128 tile of accumulator register v of block (p, q)
__device__ inline int acc_row2(int p, int v) {
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    return (w & 1) * 64 + 16 * p + (l >> 4) + 4 * v;
}
__device__ inline int acc_col2(int q) {
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    return (w >> 1) * 64 + 16 * q + (l & 15);
}

}  // namespace mg
}  // namespace lsdd
