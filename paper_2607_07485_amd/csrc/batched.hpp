// Batched, tiled FP64 dense kernels for the local problems of many
// aggregates at once (variable sizes).  A matrix "view" is a column-major
// block at base + off with leading dimension ld; every operation runs tile
// jobs (64 x 64) of all views of the batch in the same launch, the
// contractions on the FP64 matrix cores.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace lsdd {

struct View {
    int64_t off;   // offset of element (0, 0) from the base pointer
    int32_t ld;    // leading dimension
    int32_t rows;
    int32_t cols;
    int32_t pad;
};

// Host-side planner: owns small device arrays reused between launches.
struct Batched {
    hipStream_t st = nullptr;
    View* d_slot[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t slot_cap = 0;
    void* (*alloc)(void* ctx, size_t bytes) = nullptr;
    void (*release)(void* ctx, void* p) = nullptr;
    void* ctx = nullptr;

    // copy views into device slot 0, 1 or 2 (grown on demand) and return it
    View* put(int slot, const std::vector<View>& v);
    void free_all();

    // Cholesky A = L L^T (lower, in place) of every square view of `a`;
    // minpiv[b] receives the smallest pivot d_j of view b (<= 0: failure).
    void potrf(double* base, const std::vector<View>& a, double* d_minpiv);
    // Diagonally pivoted Cholesky of the trailing block of every square view:
    // indices lead[b] .. rows-1 of view b are eliminated, each time the one with
    // the largest remaining diagonal entry (lowest index among equal ones), until
    // that entry is at most d_tol[b]; rank[b] receives the number eliminated.
    // Pivots are swapped into place symmetrically across the whole view, so the
    // leading block stays where it is and the rows lead[b] .. lead[b]+rank-1 of
    // the coupling block are the pivot rows.  On return the first rank[b]
    // columns of the trailing block hold the factor (lower triangle).  Only the
    // lower triangle of the view is read and kept consistent.  d_perm (optional,
    // device, sum of rows - lead entries in view order): the trailing index at each
    // trailing position on return; with it, ties between equal diagonal entries go
    // to the lowest original index.
    void pstrf_trailing(double* base, const std::vector<View>& a, const std::vector<int32_t>& lead,
                        const double* d_tol, std::vector<int32_t>& rank, int32_t* d_perm = nullptr);
    // B <- L^{-1} B (trans = false) or B <- L^{-T} B (trans = true) with L the
    // lower triangle of the square view l[b] and B the view b[b] (rows = n).
    // lower_b (forward only): B is lower triangular (e.g. the identity), so
    // column tiles right of the current diagonal tile are skipped.
    void trsm(const double* lbase, const std::vector<View>& l, double* bbase, const std::vector<View>& b,
              bool trans, bool lower_b = false);
    // C_out = beta * C_in - alpha * A^T B for views (A: K x M, B: K x N,
    // C: M x N).  beta = 0 ignores C_in.  tri_k: A and B are lower triangular,
    // so the K loop of output tile (i, j) starts at tile max(i, j).  sym: the
    // result is symmetric (A = B, beta = 0): only lower tiles are computed and
    // each is also stored mirrored.  f32: the product runs on the FP32 matrix
    // cores (operands rounded to FP32, FP32 accumulation), C stays FP64.
    void gemm_tn(const double* abase, const std::vector<View>& a, const double* bbase, const std::vector<View>& b,
                 const double* cinbase, const std::vector<View>& cin, double beta, double* coutbase,
                 const std::vector<View>& cout, double alpha, bool tri_k = false, bool sym = false,
                 bool f32 = false);
    // In-place transpose of square views.
    void transpose(double* base, const std::vector<View>& a);
};

}  // namespace lsdd
