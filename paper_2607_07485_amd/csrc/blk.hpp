// Launchers of the block (multi right-hand side) cycle kernels and of the
// segmented PCG kernels (implemented in blk.hip).  Block vectors hold NRB
// right-hand sides interleaved per DOF: entry (d, k) at d * NRB + k.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsdd {

constexpr int NRB = 8;   // right-hand sides per block

// ---------------------------------------------------------------- cycle, block vectors
// lanes per row of the CSR kernels: 4, 8 or 16 (lane = nonzero slot, all NRB
// right-hand sides per lane) or 32 or 64 (lane = (nonzero slot, right-hand side));
// residual rows of a supernode-blocked level by supernode row blocks (blk, rows, out
// as in launch_sup_resid_blocks; scol/scoff: the shared column lists), blocks of NRB
// right-hand sides, 4 / 8 / 16 lanes per row block
template <typename T>
void launch_sup_resid_blocks_b(int64_t nblk, const int32_t* blk, const int32_t* rows, const int64_t* rowptr,
                               const int32_t* scol, const int64_t* scoff, const T* val, const T* x, const T* r, T* out,
                               bool x_zero, int lanes, hipStream_t st);
// scoff != NULL: shared per-supernode column lists, as in launch_csr_resid_rows
template <typename T>
void launch_csr_resid_rows_b(int64_t nrows, const int32_t* rows, const int64_t* rowptr, const int32_t* col,
                             const T* val, const T* x, const T* r, T* out, bool x_zero, int lanes, hipStream_t st,
                             const int64_t* scoff = nullptr);
template <typename T>
void launch_csr_spmv_b(int64_t n, const int64_t* rowptr, const int32_t* col, const T* val, const T* x, T* y,
                       const T* r_minus, int lanes, hipStream_t st, const int64_t* scoff = nullptr);
template <typename T>
void launch_sub_symv_b(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                       const T* tiles, const T* rloc, const int64_t* scr_off, T* scr, int chl, hipStream_t st);
// the block finalize from the single-vector finalize's address table (int4 per entry);
// accumulates into x
template <typename T>
void launch_sub_finalize_tab_b(int64_t r0, int64_t r1, const int32_t* tab, const T* scr, const int32_t* sub_dofs,
                               T* x, int fl, hipStream_t st);
template <typename T>
void launch_sub_finalize_b(int64_t r0, int64_t r1, const int32_t* pos_sub, const int64_t* sub_off,
                           const int64_t* scr_off, const T* scr, const int32_t* sub_dofs, T* x, bool accumulate,
                           int chl, int fl, hipStream_t st);
template <typename T>
void launch_restrict_b(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                       const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* t, T* rc,
                       hipStream_t st);
template <typename T>
void launch_prolong_b(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                      const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                      hipStream_t st);

// ---------------------------------------------------------------- small overlaps (NR = 1 or NRB)
constexpr int SMALL_M = 64;   // overlaps and aggregates up to this size use the kernels below

// x[Omega_s] += A_Omega_s^{-1} rloc[Omega_s] for the sweep-order subdomains s0 .. s0+n_sub-1
// (packed lower inverses at pk + pk_off[s]; rloc and x hold NR interleaved vectors);
// max_m (1 .. SMALL_M) bounds |Omega_s| over the launch and sizes its LDS.  fact: the
// packed triangles are lower-triangular factors X with A_Omega^{-1} = X^T X
template <typename T, int NR>
void launch_small_sub(int64_t s0, int64_t n_sub, const int64_t* sub_off, const int32_t* sub_dofs,
                      const int64_t* pk_off, const T* pk, const T* rloc, T* x, int max_m, hipStream_t st,
                      bool fact = false);
// rc[c] = Z_i[:, c - coff_i]^T t[omega_i] for every coarse DOF c of an aggregate i
// with agg_of_c[c] = i (agg_of_c[c] < 0: skipped)
template <typename T, int NR>
void launch_restrict_small(int64_t nc, const int32_t* agg_of_c, const int64_t* agg_ptr, const int32_t* agg_dofs,
                           const int64_t* zoff, const int64_t* coff, const T* Zc, const T* t, T* rc, hipStream_t st);
// x[agg_dofs[p]] += Z_i[p - agg_ptr_i, :] ec[coff_i ..] for aggregate entries p with agg_of_p[p] = i
template <typename T, int NR>
void launch_prolong_small(int64_t na, const int32_t* agg_of_p, const int64_t* agg_ptr, const int32_t* agg_dofs,
                          const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                          hipStream_t st);

// B[d * NRB + k] = k < nr ? b[k * ldb + d] : 0 (d < n); and the inverse copy
void launch_gather_rhs(int64_t n, int32_t nr, const double* b, int64_t ldb, double* B, hipStream_t st);
void launch_scatter_sol(int64_t n, int32_t nr, const double* X, double* x, int64_t ldx, hipStream_t st);

// ---------------------------------------------------------------- segmented PCG
// A "segment" is a contiguous DOF range of the level-0 vector (one problem
// instance); every (segment, right-hand side) pair i = seg * NR + k runs its own
// CG recurrence.  Reductions use a fixed block table (segment, DOF range) and
// add the block partials in block order, so every scalar is reproducible.
struct SegTable {
    int32_t n_seg = 0;
    int32_t n_blk = 0;
    const int32_t* blk_seg = nullptr;   // [n_blk]
    const int64_t* blk_lo = nullptr;    // [n_blk] first DOF
    const int64_t* blk_hi = nullptr;    // [n_blk] one past the last DOF
    const int32_t* seg_blk = nullptr;   // [n_seg + 1] blocks of segment s
};

// out0[i] = <a0, b0>_i and, when a1 != NULL, out1[i] = <a1, b1>_i;
// part holds 2 * n_blk * NR doubles
void launch_seg_dot(const SegTable& t, int nr, const double* a0, const double* b0, const double* a1,
                    const double* b1, double* part, double* out0, double* out1, hipStream_t st);
// state of the recurrences: act (1 = still iterating), iters, relres; it_flag[0]
// (iteration counter) and it_flag[1] (breakdown flag) are cleared
void launch_pcg_init(int n_s, const double* bb, int32_t* act, int32_t* iters, double* relres, int32_t* it_flag,
                     hipStream_t st);
// alpha_i = rz_i / pq_i for active pairs (0 otherwise); flag[0] = 1 on breakdown
void launch_pcg_alpha(int n_s, const int32_t* act, const double* rz, const double* pq, double* alpha,
                      int32_t* flag, hipStream_t st);
// x += alpha p, r -= alpha q on active pairs; rr_i = <r, r>_i (fused)
void launch_pcg_update_xr(const SegTable& t, int nr, const int32_t* act, const double* alpha, const double* p,
                          const double* q, double* x, double* r, double* part, double* rr, hipStream_t st);
// it_dev[0] += 1; converged pairs (rr <= tol2 * bb) leave the active set at that
// iteration; count[0] = number of active pairs; flag[0] = 1 on a non-finite residual
void launch_pcg_check(int n_s, int32_t* it_dev, double tol2, const double* bb, const double* rr, int32_t* act,
                      int32_t* iters, double* relres, int32_t* count, int32_t* flag, hipStream_t st);
// beta_i = (rz_new_i - rzold_i) / rz_i (rzold = NULL: standard beta); rz_i <- rz_new_i
void launch_pcg_beta(int n_s, const int32_t* act, const double* rz_new, const double* rz_old_dot, double* rz,
                     double* beta, int32_t* flag, hipStream_t st);
// p = z + beta p on active pairs
void launch_pcg_update_p(const SegTable& t, int nr, const int32_t* act, const double* beta, const double* z,
                         double* p, hipStream_t st);
// x = 0 and r = b on every pair (r, x block or single vectors)
void launch_pcg_start(int64_t len, const double* b, double* r, double* x, hipStream_t st);

}  // namespace lsdd
