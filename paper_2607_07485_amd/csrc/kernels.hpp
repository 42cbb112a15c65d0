// Launchers of the HIP kernels (implemented in kernels.hip).  All take the
// stream last and enqueue asynchronously.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "batched.hpp"
#include "consts.hpp"
#include "symv.hpp"

namespace lsdd {

struct LocalArgs {
    // per aggregate (batch-relative index b, aggregate a = first + b)
    int32_t first;                 // first aggregate of the batch
    const int32_t* agg_list;       // optional: aggregate of batch entry b (assembly re-runs)
    const int64_t* sub_ptr;        // Omega offsets into sub_dofs (aggregate order)
    const int32_t* sub_dofs;
    const int64_t* agg_ptr;        // omega sizes = agg_ptr[a+1]-agg_ptr[a]
    const int64_t* cl_ptr;         // elements of cl(omega_a)
    const int32_t* cl_elems;
    const int64_t* clpos_off;      // per cl entry: offset of its n_e local positions
    const int32_t* clpos;
    const int32_t* mult;           // per element
    const int64_t* elem_ptr;       // element supports (for n_e)
    const int64_t* blk_off;        // element block offsets (n_e^2 each, row-major)
    const double* blocks;
    const int64_t* rowptr;         // CSR of A_l
    const int32_t* col;
    const double* val;
    // workspace (batch-relative offsets)
    const int64_t* ws_off;         // per batch entry: offset of its m x m slots
    double* w1;                    // A~_Omega, later sorted eigenvectors / Z
    double* w2;                    // A_Omega, then its Cholesky factor
    const int64_t* sq_off;         // per batch entry: offset of its nw x nw slots
    double* s_buf;                 // S~, then C
    double* v_buf;                 // Jacobi eigenvectors
    const int64_t* t_off;          // per batch entry: tridiagonal data + inverse-iteration scratch
    double* t_buf;
    // outputs
    const int64_t* inv_off;        // aggregate order: offset of A_Omega^{-1} (m x m)
    double* inv;
    const int64_t* zst_off;        // aggregate order: staging Z (nw x k, row-major)
    double* zst;
    const int64_t* mu_off;         // = agg_ptr (sorted mu per aggregate)
    double* mu;
    int32_t* k_out;
    int32_t* status;               // 0 ok, 2 A_Omega not SPD
    // parameters
    int32_t modes_fixed;
    double thr;                    // 1 / tau_cut
    const double* thr_agg;         // optional per-aggregate 1 / tau_cut (batched instances)
    double band_tol, cluster_tol;
    int32_t trd_min;               // > 0: aggregates with nw >= trd_min were reduced by the blocked path
};

// Blocked multi-workgroup tridiagonalisation (trd.hip) of the batch entries
// d_big[0 .. sizes.size()) (sizes = their nw, each > 2 TRD_NB + 1); leaves the
// same d, e, tau and reflectors as the single-workgroup reduction of k_local_eig.
constexpr int TRD_NB = 32;
void launch_local_tridiag_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                  hipStream_t st);
// Retained eigenvectors of the tridiagonal matrices of the same entries by
// inverse iteration, ceil(k / 64) workgroups per entry (after the mode-count
// phase of k_local_eig); iw + iw_off[i] is entry i's scratch of
// ceil(k_i / 64) * (INVIT_SLOTS n_i + 4096) doubles.
void launch_local_invit_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                const std::vector<int32_t>& ks, const int64_t* d_iw_off, double* iw, hipStream_t st);
// Back-transformation of the retained eigenvectors of the same entries (after
// the eigenvalue and inverse-iteration phases).
void launch_local_backtransform_blocked(const LocalArgs& a, const int32_t* d_big, const std::vector<int32_t>& sizes,
                                        hipStream_t st);

// Element Gram factors from eigendecompositions: Jacobi in LDS for blocks up to 48,
// the tridiagonal route above; n_max = largest block, scratch of
// elem_eig_scratch_stride(n_max) doubles per element.
void launch_elem_eig(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                     double* G, int32_t* ranks, int32_t* status, double* scratch, int64_t scratch_stride,
                     double rank_rtol, double spsd_tol, int64_t n_max, hipStream_t st);
int64_t elem_eig_scratch_stride(int64_t n_max);

// CSR values += sum_T f_T R_T^T A_T R_T (f = factor, NULL = 1); d2e lists the
// (element, local index) pairs of every DOF, elements ascending; wave_rows: one
// wave per row (long element rows of coarse levels), same summation order
void launch_elem_pchol(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                       double* G, int32_t* ranks, int32_t* status, double* scratch, int64_t scratch_stride,
                       double rank_rtol, double spsd_tol, hipStream_t st);
void launch_assemble_rows(int64_t n, const int64_t* d2e_ptr, const int32_t* d2e_elem, const int32_t* d2e_loc,
                          const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* blk_off,
                          const double* blocks, const double* factor, const int64_t* rowptr, const int32_t* col,
                          double* val, hipStream_t st, bool wave_rows = false);
// factor[e] = theta[e] / theta0[e] (theta0 NULL: theta[e])
void launch_theta_factor(int64_t n, const double* theta, const double* theta0, double* factor, hipStream_t st);
// Element-batch operator apply: y = A x (r_minus NULL) or y = r_minus - A x with
// A = sum_e R_e^T A_e R_e from the packed lower triangles of the A_e (tri at
// tri_off[e]; n_max the largest element, <= 128), through a per-element buffer ybuf
// (one entry per elem_dofs entry) summed per DOF in ascending element order
// (d2e_ptr over the DOFs, e2y the elem_dofs position of each (DOF, element) pair).
template <typename T, typename V>
void launch_elem_apply(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* tri_off,
                       const V* tri, int n_max, const T* x, V* ybuf, int64_t n, const int64_t* d2e_ptr,
                       const int32_t* e2y, const T* r_minus, T* y, hipStream_t st);
// packed lower triangles of factor[e] * A_e (factor NULL: 1), FP64 and optionally FP32
void launch_pack_elem_tri(int64_t n_elem, const int64_t* elem_ptr, const int64_t* blk_off, const double* blocks,
                          const double* factor, const int64_t* tri_off, double* tri, float* tri32, hipStream_t st);
// Black-box Gram factor rows as elements: G_e = [g; 0] and A_e = g^T g for the row g
// of element e (values at val + src_off[e], elem_ptr giving its length).
void launch_gram_csr_rows(int64_t n_elem, const int64_t* elem_ptr, const int64_t* src_off, const int64_t* blk_off,
                          const double* val, double* G, double* blocks, hipStream_t st);
// Gram rows G_e (row-major n_e x n_e at blk_off[e]) from pivoted Cholesky factors
// in pivot order: G_e(k, perm[i]) = L_e(i, k) for k < rank[e], zero elsewhere.
// perm_off: elem_ptr of the elements (perm of element e at perm_off[e] - perm_off[0]).
void launch_gram_rows(int64_t n_elem, const int64_t* perm_off, const int64_t* blk_off, const double* L,
                      const int32_t* perm, const int32_t* rank, double* G, hipStream_t st);
// blocks of element e *= scale[e]
void launch_scale_blocks(int64_t n_elem, const int64_t* blk_off, const double* scale, double* blocks, hipStream_t st);
// out[e] = scale * sum_k u_{k,e}^T B_e v_{k,e} over nrhs vectors at stride ld
void launch_elem_bilinear(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs, const int64_t* blk_off,
                          const double* blocks, const double* u, const double* v, int32_t nrhs, int64_t ld,
                          double scale, double* out, hipStream_t st);
// blk_off[0 .. n_elem] = prefix sums of the squared element sizes (device elem_ptr)
void launch_block_offsets(int64_t n_elem, const int64_t* elem_ptr, int64_t* blk_off, hipStream_t st);

// Allocation-free entry points (noalloc.hip): the device address, on the current
// device, of a static scratch array of 2 (NOALLOC_MAX_ELEM + 1) int64 entries
// (16 MiB), looked up once per device and shared by every call on that device.
constexpr int64_t NOALLOC_MAX_ELEM = int64_t(1) << 20;
hipError_t noalloc_scratch(int64_t** out);

void launch_local_assemble(int32_t nbatch, const LocalArgs& a, int32_t max_m, hipStream_t st);
// max_nw: largest |omega| of the batch (<= 4096)
void launch_local_eig(int32_t nbatch, const LocalArgs& a, int32_t max_nw, int first_phase, int last_phase,
                      hipStream_t st);
void launch_stage_z(int32_t nbatch, const LocalArgs& a, hipStream_t st);
void launch_views_max_diag(int32_t nv, const double* base, const View* v, double* out, hipStream_t st);
void launch_views_add_diag(int32_t nv, double* base, const View* v, const double* delta, hipStream_t st);
void launch_views_symmetrize(int32_t nv, double* base, const View* v, hipStream_t st);
void launch_views_identity(int32_t nv, double* base, const View* v, hipStream_t st);

void launch_z_compact(int32_t n_agg, const int64_t* agg_ptr, const int32_t* k, const int64_t* zst_off,
                      const double* zst, const int64_t* zoff, double* Z, double* Zc, float* Zc32, hipStream_t st);

// Galerkin products run as batched matrix-core contractions over stacked
// interpolation rows: for coarse group g with members e (fine element blocks
// F_e, n_e x n_e row-major) and stacked P_g = [P_e] (R_g x c_g),
// Y_e = F_e P_e, then A_g = Y^T Y (level 0, F_e = Gram factor G_e) or
// A_g = P_g^T Y (F_e = A_e).  This kernel writes P_g.
struct PstArgs {
    int32_t g0, n_groups;          // groups g0 .. g0 + n_groups - 1
    const int64_t* cptr;           // coarse group supports (sizes c_g)
    const int64_t* mem_ptr;        // members of group g
    const int32_t* mem_elems;
    const int64_t* felem_ptr;      // fine element supports (n_e)
    const int64_t* pm_off;         // per member entry: offset of its n_e map entries
    const int64_t* pm_zrow;        // per (member, local dof): Z row offset (-1: no mode)
    const int32_t* pm_k;           //   modes of its aggregate
    const int32_t* pm_col;         //   column offset of its aggregate in the group support
    const double* Z;
    const int64_t* pst_off;        // per group of the launch: offset of P_g
    const int64_t* rows;           //   R_g
    double* pst;
};
void launch_build_pst(const PstArgs& g, hipStream_t st);

// D = A[off:off+n, off:off+n] (column-major n x n; D must be zeroed first)
void launch_dense_from_csr(int64_t off, int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                           double* D, hipStream_t st);

void launch_to_f32(int64_t n, const double* a, float* b, hipStream_t st);
void launch_to_f64(int64_t n, const float* a, double* b, hipStream_t st);

// ---------------------------------------------------------------- solve
// lanes per row: 8, 16, 32 or 64.  V: value type (T, or double with T = float:
// FP64 operator entries applied to FP32 vectors with FP64 sums)
// scoff != NULL: col holds one column list per supernode and row p's list starts at
// col[scoff[p]] (rows of a supernode share their columns); else the CSR's own col
template <typename T, typename V = T>
void launch_csr_resid_rows(int64_t nrows, const int32_t* rows, const int64_t* rowptr, const int32_t* col,
                           const V* val, const T* x, const T* r, T* out, bool x_zero, int lanes, hipStream_t st,
                           const int64_t* scoff = nullptr);
// residual rows of a supernode-blocked level by row blocks of one supernode (blk:
// per block the first list position and the row count, 1..8; rows, out: the whole
// list); scol/scoff as the shared column lists of launch_csr_resid_rows; waves (1,
// 2 or 4) per block
template <typename T, typename V = T>
void launch_sup_resid_blocks(int64_t nblk, const int32_t* blk, const int32_t* rows, const int64_t* rowptr,
                             const int32_t* scol, const int64_t* scoff, const V* val, const T* x, const T* r, T* out,
                             bool x_zero, int waves, hipStream_t st);
template <typename T, typename V = T>
void launch_csr_spmv(int64_t n, const int64_t* rowptr, const int32_t* col, const V* val, const T* x, T* y,
                     const T* r_minus, int lanes, hipStream_t st, const int64_t* scoff = nullptr);
// chl: tiles per work item (1..8); the scratch layout depends on it
template <typename T>
void launch_sub_symv(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                     const T* tiles, const T* rloc, const int64_t* scr_off, T* scr, int chl, hipStream_t st);
// x[sub_dofs[t]] (+)= sum of the partials of entry t, for t in [r0, r1); sub_dofs NULL = identity;
// fl: threads per entry (8 or 32)
template <typename T>
void launch_sub_finalize(int64_t r0, int64_t r1, const int32_t* pos_sub, const int64_t* sub_off,
                         const int64_t* scr_off, const T* scr, const int32_t* sub_dofs, T* x, bool accumulate,
                         int chl, int fl, hipStream_t st);
// the same (accumulating) from a table of 4 int32 per entry t (16-byte aligned):
// {row-part address of chunk 0, scr_off + rowpart_off(nt) * 64 + J * 64 + l, J, nch | nt << 16}
template <typename T>
void launch_sub_finalize_tab(int64_t r0, int64_t r1, const int32_t* tab, const T* scr, const int32_t* sub_dofs, T* x,
                             int fl, hipStream_t st);
// mixed cycle: y = X^T (X r) with FP32 factor tiles in one pass, FP64 sums; items =
// (subdomain, whole tile row) pairs; partials in the layout of launch_sub_symv for chl.
// stash: tiles of each row kept in LDS between the two products (0 .. SUB_FACT_MAX_STASH;
// 16 KB each, all work items of the launch get the same allocation)
constexpr int SUB_FACT_MAX_STASH = 8;
void launch_sub_fact(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                     const float* tiles, const float* rloc, const int64_t* scr_off, float* scr, int chl, int stash,
                     hipStream_t st);
// scratch entries for a subdomain of size m; append its work items (s, tile row, chunk)
int64_t sub_symv_scratch_len(int64_t m, int chl);
void sub_symv_items(int32_t s, int64_t m, int chl, std::vector<int32_t>& items);
// packed lower triangles of the inverses of the aggregates with pk_off[a] >= 0
void launch_pack_small(int32_t n_agg, const int64_t* sub_ptr, const int64_t* inv_off, const double* inv,
                       const int64_t* pk_off, double* pk, float* pk32, hipStream_t st);
void launch_pack_tiles(int32_t n_agg, const int64_t* sub_ptr, const int64_t* inv_off, const double* inv,
                       const int64_t* tp_off, double* tiles, float* tiles32, hipStream_t st);
// restriction items: (aggregate, first of 16 columns); prolongation items: (aggregate, first of 256 rows)
template <typename T>
void launch_restrict(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                     const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* t, T* rc,
                     hipStream_t st);
template <typename T>
void launch_prolong(int64_t n_items, const int32_t* items, const int64_t* agg_ptr, const int32_t* agg_dofs,
                    const int64_t* zoff, const int32_t* k, const int64_t* coff, const T* Zc, const T* ec, T* x,
                    hipStream_t st);
template <typename T>
void launch_zero(int64_t n, T* x, hipStream_t st);

// PCG helpers (FP64).  `partials` holds at least 1024 doubles.
void launch_dot(int64_t n, const double* a, const double* b, double* partials, double* out, hipStream_t st);
// x += alpha p; r -= alpha q with alpha = s[0] / s[1]; out = ||r||^2
void launch_update_xr(int64_t n, const double* s_num, const double* s_den, const double* p, const double* q,
                      double* x, double* r, double* partials, double* out_rr, hipStream_t st);
// p = z + (s_num / s_den) p
void launch_update_p(int64_t n, const double* s_num, const double* s_den, const double* z, double* p,
                     hipStream_t st);
void launch_copy(int64_t n, const double* a, double* b, hipStream_t st);
// Timing events the next launch of the subdomain product records at the kernel's own
// start and end (hipExtLaunchKernel), instead of separate event packets around it;
// take_launch_events hands them to that launch once.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool take_launch_events(hipEvent_t* start, hipEvent_t* stop);
// y += a x
void launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t st);
void launch_check_finite(int64_t n, const double* a, int32_t* flag, hipStream_t st);

}  // namespace lsdd
