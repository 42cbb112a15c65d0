// Host driver of the LS-AMG-DD library: hierarchy construction (integer work
// on the host, numerics in HIP kernels), the V-cycle, PCG and the C-ABI.
#include "lsdd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cfloat>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "graph.hpp"
#include "kernels.hpp"
#include "blk.hpp"

namespace {

thread_local std::string g_err;
lsdd_alloc_fn g_alloc = nullptr;
lsdd_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;

struct Error : std::runtime_error {
    lsdd_status code;
    Error(lsdd_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess)                                                                      \
            throw Error(LSDD_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));               \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// LSDD_VERBOSE=1 prints setup phase timings to stderr.
bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("LSDD_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}

// Local spectral problems with at least this many aggregate DOFs are reduced to
// tridiagonal form by the blocked multi-workgroup path (0: every reduction in
// one workgroup).
int32_t trd_min(int32_t param) {
    if (param < 0) return 0;
    if (param == 0) return 192;
    return std::max<int32_t>(param, 2 * lsdd::TRD_NB + 2);
}

void vlog(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void vlog(const char* fmt, ...) {
    if (!verbose()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[lsdd] ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
    va_end(ap);
}

}  // namespace

namespace lsdd {

// Device memory owned by one hierarchy; released in one go.
struct Arena {
    std::vector<void*> ptrs;
    void* get(size_t bytes) {
        if (bytes == 0) bytes = 8;
        bytes = (bytes + 255) & ~size_t(255);
        void* p = nullptr;
        if (g_alloc) {
            p = g_alloc(bytes, g_alloc_ctx);
            if (!p) throw Error(LSDD_E_NOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) throw Error(LSDD_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
        }
        ptrs.push_back(p);
        return p;
    }
    template <typename T>
    T* alloc(size_t count) { return static_cast<T*>(get(count * sizeof(T))); }
    template <typename T>
    T* upload(const std::vector<T>& v, hipStream_t st) {
        T* p = alloc<T>(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        return p;
    }
    void release(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it == ptrs.end()) return;
        if (g_free) g_free(p, g_alloc_ctx);
        else (void)hipFree(p);
        ptrs.erase(it);
    }
    void clear() {
        for (void* p : ptrs) {
            if (g_free) g_free(p, g_alloc_ctx);
            else (void)hipFree(p);
        }
        ptrs.clear();
    }
};

template <typename T>
std::vector<T> download(const T* d, size_t count, hipStream_t st) {
    std::vector<T> h(count);
    if (count) {
        HIPCHK(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return h;
}

template <typename T>
struct VecSet {
    T* r = nullptr;
    T* x = nullptr;
    T* t = nullptr;
    T* rloc = nullptr;
    T* scr = nullptr;
};

struct Level {
    int32_t level = 0;
    int64_t n = 0;
    int64_t nnz = 0;
    std::vector<int64_t> inst_off;     // DOF range of every problem instance (contiguous)
    ElemList el;
    std::vector<int64_t> blk_off;
    int64_t* d_elem_ptr = nullptr;
    int32_t* d_elem_dofs = nullptr;
    int64_t* d_blk_off = nullptr;
    double* d_blocks = nullptr;
    // assembled operator
    Csr pat;
    int lanes = 16;                    // CSR lanes per row, single vectors (4, 8, 16, 32 or 64)
    int lanes_b = 8;                   // CSR lanes per row, blocks of NRB vectors (4, 8, 16, 32 or 64)
    int chl = SUB_MAX_CHUNK;           // tiles per subdomain-kernel work item
    int fl = 8;                        // threads per DOF in the subdomain finalize
    int64_t* d_rowptr = nullptr;
    int32_t* d_col = nullptr;
    double* d_val = nullptr;
    int64_t* d_d2e_ptr = nullptr;     // level 0: DOF -> (element, local index), kept for re-assembly
    int32_t* d_d2e_elem = nullptr;
    int32_t* d_d2e_loc = nullptr;
    // level 0: element-batch operator apply from the packed lower triangles of the
    // element blocks (built when the autotuner first times it)
    double* d_etri = nullptr;
    float* d_etri32 = nullptr;
    int64_t* d_etri_off = nullptr;
    int32_t* d_e2y = nullptr;         // per (DOF, element) pair: its elem_dofs position
    double* d_ebuf = nullptr;         // per elem_dofs entry: (A_e x_e)_j
    float* d_ebuf32 = nullptr;
    int64_t etri_len = 0;
    int e_nmax = 0;
    int eapply = 0;                   // 1: full products of the level from the element triangles
    // supernode-blocked pattern: the rows of a supernode share one column list
    int32_t* d_scol = nullptr;        // the lists, one per supernode
    int64_t* d_scoff = nullptr;       // per row: start of its supernode's list
    double sup_ib = 4.0;              // column-index bytes per entry read from HBM with the lists
    int sup = 0;                      // 1: single-vector CSR kernels read the shared lists; 2, 3, 4: and
                                      // the sweep residuals run by supernode row blocks, 1, 2 or 4
                                      // waves per block
    // row blocks of the sweep lists: (first list position, rows 1..8) per run of
    // list entries of one supernode, grouped by colour
    int32_t* d_rblk = nullptr;
    std::vector<int64_t> color_rblk0;
    float* d_val32 = nullptr;
    // level-0 Gram factors
    double* d_G = nullptr;
    std::vector<int32_t> ranks;
    // supernodes
    std::vector<int32_t> node_of_dof;
    int32_t n_super = 0;
    // coarsening
    bool coarsest = false;
    std::vector<int32_t> agg_of_dof;
    Closure cl;
    std::vector<int32_t> colors;
    int32_t n_colors = 0;
    std::vector<int32_t> k;
    std::vector<int64_t> zoff, coff;
    int64_t* d_agg_ptr = nullptr;
    int32_t* d_agg_dofs = nullptr;
    int64_t* d_zoff = nullptr;
    int32_t* d_k = nullptr;
    int64_t* d_coff = nullptr;
    double* d_Z = nullptr;        // row-major Z_i (Galerkin products, export)
    double* d_Zc = nullptr;       // column-major Z_i (transfers)
    float* d_Zc32 = nullptr;
    int32_t* d_ritems = nullptr;  // restriction work items
    int32_t* d_pitems = nullptr;  // prolongation work items
    int64_t n_ritems = 0, n_pitems = 0;
    double* d_mu = nullptr;
    // smoother, sweep order (colour-major, aggregate index within a colour)
    std::vector<int32_t> sweep;
    std::vector<int64_t> sw_sub_off;
    std::vector<int64_t> color_row0, color_item0;
    // inside a colour: large overlaps (tiled product) first, then small ones (packed, one wave each)
    std::vector<int64_t> color_rmid;  // first row of the colour's small overlaps
    std::vector<int32_t> color_sub0;  // first sweep position of the colour
    std::vector<int32_t> color_smid;  // first small sweep position of the colour
    int32_t small_m = 1;                  // largest small overlap (sizes the small kernel's LDS)
    std::vector<double> color_pk;     // packed entries of the colour's small overlaps
    int64_t* d_sw_pk_off = nullptr;   // packed-inverse offset of each small subdomain (sweep order)
    double* d_pk = nullptr;
    float* d_pk32 = nullptr;
    int32_t* d_agg_of_c = nullptr;    // coarse DOF -> aggregate for small aggregates (-1: large)
    int32_t* d_agg_of_p = nullptr;    // aggregate entry -> aggregate for small aggregates (-1: large)
    int64_t n_aggent = 0;             // sum |omega_i|
    std::vector<double> color_m2, color_m, color_nnz;   // sums of |Omega|^2, |Omega|, row nnz per colour
    int64_t* d_sw_sub_off = nullptr;
    int32_t* d_sw_sub_dofs = nullptr;
    int32_t* d_sw_sub_dofs_w = nullptr;   // RAS: the same with interface entries = -1
    int32_t smoother = 0;                 // 0 multiplicative Schwarz, 1 RAS, 2 block Jacobi
    int64_t* d_sw_tp_off = nullptr;   // packed-tile offset of each subdomain (sweep order)
    int32_t* d_items = nullptr;       // (subdomain, tile row), grouped by colour
    int32_t* d_row_items = nullptr;   // mixed cycle: (subdomain, whole tile row), grouped by colour
    std::vector<int64_t> color_ritem0;
    std::vector<int> color_stash;     // mixed cycle: factor tiles per row kept in LDS, per colour
    int fact_stash = 1;               // 0: the factor product re-reads every tile through the caches
    int32_t* d_pos_sub = nullptr;     // sweep-order subdomain of every Omega entry
    int64_t* d_scr_off = nullptr;     // per subdomain: offset of its partial-sum scratch
    int32_t* d_fin_tab = nullptr;     // per overlap entry: its partial-sum addresses (4 int32)
    // coarsest level as one packed symmetric "subdomain"
    // terminal blocks: the instances whose hierarchy ends on this level (every
    // instance present on the coarsest level), each solved with its dense inverse
    std::vector<int32_t> term;        // instance ids
    int64_t term_len = 0;             // DOFs in terminal blocks (entries, instance order)
    int64_t c_scr_len = 0;            // partial-sum entries of the terminal product
    int c_chl = SUB_MAX_CHUNK;        // tiles per work item of the terminal product
    double c_entries = 0.0;           // sum n_i (n_i + 1) / 2 over the blocks
    int64_t* c_sub_off = nullptr;     // entry ranges of the blocks
    int64_t* c_tp_off = nullptr;
    int64_t* c_scr_off = nullptr;
    int32_t* c_pos = nullptr;         // entry -> block
    int32_t* c_dofs = nullptr;        // entry -> DOF (NULL: the blocks cover the level in order)
    int32_t* c_items = nullptr;
    int64_t c_nitems = 0;
    double* c_tiles = nullptr;
    double* d_inv = nullptr;          // full inverses during setup only
    double* d_tiles = nullptr;        // packed lower tiles of A_Omega^{-1}
    float* d_tiles32 = nullptr;
    double* d_X = nullptr;            // full factors X = L^{-1} of A_Omega during setup (precision 2)
    float* d_tfac32 = nullptr;        // packed lower tiles of X (FP32), A_Omega^{-1} = X^T X
    float* d_pkfac32 = nullptr;       // packed lower triangles of X for the small overlaps (FP32)
    int64_t inv_len = 0, tiles_len = 0;
    // vectors: [0] single vectors, [1] blocks of NRB right-hand sides (allocated on first use)
    VecSet<double> v64[2];
    VecSet<float> v32[2];
    double* cr64[2] = {nullptr, nullptr};   // FP64 staging for the FP32 coarsest solve
    double* cx64[2] = {nullptr, nullptr};
    int64_t rloc_len = 0;                   // gathered subdomain residual entries (sum |Omega_i|)
    int64_t scr_len = 0;                    // partial-sum entries of the subdomain product
    std::vector<double> color_scr;          // partial-sum entries per colour
};

// Per-kernel-class HIP-event timing on the hierarchy's stream, with the
// algorithmic bytes of each traced launch (enabled by lsdd_trace).
struct Trace {
    struct Agg {
        std::string name;
        int64_t launches = 0;
        double ms = 0.0;
        double bytes = 0.0;
    };
    struct Pend {
        int idx;
        hipEvent_t a, b;
        double bytes;
    };
    bool on = false;
    std::vector<Agg> agg;
    std::vector<Pend> pend;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (pool.empty()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    int index(const char* name) {
        for (size_t i = 0; i < agg.size(); ++i)
            if (agg[i].name == name) return (int)i;
        agg.push_back(Agg{name});
        return (int)agg.size() - 1;
    }
    void flush() {   // the stream must be synchronised
        for (Pend& p : pend) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
            agg[p.idx].launches++;
            agg[p.idx].ms += ms;
            agg[p.idx].bytes += p.bytes;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pend.clear();
    }
    void destroy() {
        for (Pend& p : pend) {
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pend.clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

}  // namespace lsdd

struct lsdd_hierarchy {
    int32_t cycle_prec = 0;       // 0 FP64 cycle, 1 FP32 cycle (params.precision >= 1), 2 mixed (== 2)
    lsdd::Trace tr;
    lsdd_params prm;
    hipStream_t st = nullptr;
    lsdd::Arena arena;
    std::vector<std::unique_ptr<lsdd::Level>> L;
    double setup_s = 0.0;
    // PCG work vectors: [0] single vectors, [1] blocks of NRB right-hand sides
    struct PcgBuf {
        double *B = nullptr, *X = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *rold = nullptr;
    } pb[2];
    // segments of the level-0 vector (one per problem instance) and the reduction table
    std::vector<int64_t> seg_off;
    lsdd::SegTable seg;
    int32_t nsm = 0;              // n_seg * NRB: stride of the per-pair scalar arrays
    double* sc = nullptr;         // per-pair scalars: bb rz pq rr rzn rzo alpha beta relres
    int32_t* ic = nullptr;        // act, iters (nsm each), then count, it, flag, finite-check flag
    double* part = nullptr;       // reduction partials, 2 * n_blk * NRB
    int32_t* h_ic = nullptr;      // pinned host mirror of count, it, flag
    // element coefficients the level-0 blocks were scaled with at setup (NULL: none)
    double* d_scale0 = nullptr;
    double* d_factor = nullptr;   // scratch for lsdd_update_theta
    int32_t breakdown_bits = 0;   // cause of the last PCG breakdown (k_pcg_alpha/check/beta bits)
    // hipGraph-captured halves of the PCG iteration: [block][cycle precision][half]
    bool use_graph = false;
    hipGraphExec_t gx[2][3][2] = {};
};

namespace lsdd {

namespace {

void sync(hipStream_t st) { HIPCHK(hipStreamSynchronize(st)); }

std::string breakdown_cause(int32_t bits) {
    std::string s;
    auto add = [&](const char* t) { s += (s.empty() ? "" : ", ") + std::string(t); };
    if (bits & 1) add("p^T A p <= 0 (preconditioner or operator not positive definite)");
    if (bits & 2) add("p^T A p or r^T z not finite");
    if (bits & 4) add("residual norm not finite");
    if (bits & 8) add("beta not finite");
    return s.empty() ? "unknown" : s;
}

// Device copies of a level's element supports and blocks.
void upload_elements(lsdd_hierarchy* h, Level& lv) {
    lv.d_elem_ptr = h->arena.upload(lv.el.ptr, h->st);
    lv.d_elem_dofs = h->arena.upload(lv.el.dofs, h->st);
    lv.d_blk_off = h->arena.upload(lv.blk_off, h->st);
}

// Shared column lists of a supernode-blocked pattern (every row of a supernode has
// the same columns): one list per supernode and, per row, where its list starts.
// Kept only where the lists are at most half the column indices.
void build_supernode_cols(lsdd_hierarchy* h, Level& lv) {
    std::vector<int64_t> soff(lv.n_super + 1, -1), scoff(lv.n);
    std::vector<int32_t> scol;
    int32_t prev = -1;
    for (int64_t d = 0; d < lv.n; ++d) {
        const int32_t sn = lv.node_of_dof[d];
        const int64_t a = lv.pat.ptr[d], len = lv.pat.ptr[d + 1] - a;
        if (sn != prev) {
            soff[sn] = (int64_t)scol.size();
            scol.insert(scol.end(), lv.pat.idx.begin() + a, lv.pat.idx.begin() + a + len);
            prev = sn;
        } else {
            const int64_t b = lv.pat.ptr[d - 1], lb = a - b;
            if (lb != len || !std::equal(lv.pat.idx.begin() + a, lv.pat.idx.begin() + a + len, lv.pat.idx.begin() + b))
                return;                       // not a shared pattern after all
        }
        scoff[d] = soff[sn];
    }
    if (2 * (int64_t)scol.size() > lv.nnz) return;
    lv.d_scol = h->arena.upload(scol, h->st);
    lv.d_scoff = h->arena.upload(scoff, h->st);
    lv.sup_ib = 4.0 * (double)scol.size() / (double)std::max<int64_t>(lv.nnz, 1);
    sync(h->st);
}

void assemble_operator(lsdd_hierarchy* h, Level& lv) {
    // element supports made of whole supernodes with contiguous DOF ranges (the
    // coarse levels always): the pattern is built on supernodes
    const bool blocked = assembled_pattern_blocked(lv.n, lv.el, lv.node_of_dof, lv.n_super, lv.pat);
    if (!blocked) lv.pat = assembled_pattern(lv.n, lv.el);
    lv.nnz = (int64_t)lv.pat.idx.size();
    lv.lanes = (lv.nnz > 96 * lv.n) ? 64 : 16;
    lv.lanes_b = (lv.nnz > 40 * lv.n) ? 16 : 8;
    lv.d_rowptr = h->arena.upload(lv.pat.ptr, h->st);
    lv.d_col = h->arena.upload(lv.pat.idx, h->st);
    lv.d_val = h->arena.alloc<double>(lv.nnz);
    HIPCHK(hipMemsetAsync(lv.d_val, 0, lv.nnz * sizeof(double), h->st));
    {
        // DOF -> (element, local index), elements ascending
        std::vector<int64_t> dptr(lv.n + 1, 0);
        for (int32_t d : lv.el.dofs) dptr[d + 1]++;
        for (int64_t i = 0; i < lv.n; ++i) dptr[i + 1] += dptr[i];
        std::vector<int32_t> de(lv.el.dofs.size()), dl(lv.el.dofs.size());
        std::vector<int64_t> fill(dptr.begin(), dptr.end() - 1);
        for (int64_t e = 0; e < lv.el.count(); ++e)
            for (int64_t q = lv.el.ptr[e]; q < lv.el.ptr[e + 1]; ++q) {
                int64_t t = fill[lv.el.dofs[q]]++;
                de[t] = (int32_t)e;
                dl[t] = (int32_t)(q - lv.el.ptr[e]);
            }
        int64_t* d_dptr = h->arena.upload(dptr, h->st);
        int32_t* d_de = h->arena.upload(de, h->st);
        int32_t* d_dl = h->arena.upload(dl, h->st);
        int64_t max_ne = 0;
        for (int64_t e = 0; e < lv.el.count(); ++e) max_ne = std::max(max_ne, lv.el.ptr[e + 1] - lv.el.ptr[e]);
        launch_assemble_rows(lv.n, d_dptr, d_de, d_dl, lv.d_elem_ptr, lv.d_elem_dofs, lv.d_blk_off, lv.d_blocks,
                             nullptr, lv.d_rowptr, lv.d_col, lv.d_val, h->st, max_ne > 48);
        HIPCHK(hipStreamSynchronize(h->st));
        if (lv.level == 0) {
            lv.d_d2e_ptr = d_dptr;
            lv.d_d2e_elem = d_de;
            lv.d_d2e_loc = d_dl;
        } else {
            h->arena.release(d_dptr);
            h->arena.release(d_de);
            h->arena.release(d_dl);
        }
    }
    if (h->prm.precision >= 1) {
        lv.d_val32 = h->arena.alloc<float>(lv.nnz);
        launch_to_f32(lv.nnz, lv.d_val, lv.d_val32, h->st);
    }
    if (blocked) build_supernode_cols(h, lv);
}

// Element-batch apply of level 0 (packed lower triangles of factor[e] A_e, factor =
// the theta update's ratio when one was applied).  Returns false where the level
// has no element blocks or an element above 128 DOFs.
bool build_elem_apply(lsdd_hierarchy* h, Level& lv);

void pack_elem_tri(lsdd_hierarchy* h, Level& lv) {
    launch_pack_elem_tri(lv.el.count(), lv.d_elem_ptr, lv.d_blk_off, lv.d_blocks, h->d_factor, lv.d_etri_off,
                         lv.d_etri, lv.d_etri32, h->st);
}

bool build_elem_apply(lsdd_hierarchy* h, Level& lv) {
    if (lv.d_etri) return true;
    if (lv.level != 0 || !lv.d_d2e_ptr || !lv.d_blocks) return false;
    const int64_t ne = lv.el.count();
    int64_t n_max = 0;
    std::vector<int64_t> toff(ne + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t m = lv.el.ptr[e + 1] - lv.el.ptr[e];
        n_max = std::max(n_max, m);
        toff[e + 1] = toff[e] + m * (m + 1) / 2;
    }
    if (n_max > 128 || n_max < 1) return false;
    // (DOF, element) pairs in DOF order, elements ascending: their elem_dofs positions
    std::vector<int64_t> dptr(lv.n + 1, 0);
    for (int32_t d : lv.el.dofs) dptr[d + 1]++;
    for (int64_t i = 0; i < lv.n; ++i) dptr[i + 1] += dptr[i];
    std::vector<int32_t> e2y(lv.el.dofs.size());
    std::vector<int64_t> fill(dptr.begin(), dptr.end() - 1);
    for (int64_t q = 0; q < (int64_t)lv.el.dofs.size(); ++q) e2y[fill[lv.el.dofs[q]]++] = (int32_t)q;
    Arena& ar = h->arena;
    lv.e_nmax = (int)n_max;
    lv.etri_len = toff[ne];
    lv.d_etri_off = ar.upload(toff, h->st);
    lv.d_e2y = ar.upload(e2y, h->st);
    lv.d_etri = ar.alloc<double>(lv.etri_len);
    lv.d_ebuf = ar.alloc<double>(std::max<int64_t>((int64_t)lv.el.dofs.size(), 1));
    if (h->prm.precision >= 1) {
        lv.d_etri32 = ar.alloc<float>(lv.etri_len);
        lv.d_ebuf32 = ar.alloc<float>(std::max<int64_t>((int64_t)lv.el.dofs.size(), 1));
    }
    pack_elem_tri(h, lv);
    HIPCHK(hipGetLastError());
    sync(h->st);
    vlog("level %d: element triangles, %lld entries (CSR %lld)", lv.level, (long long)lv.etri_len,
         (long long)lv.nnz);
    return true;
}

// algorithmic bytes of one full product y = A x (or r - A x): CSR rows, or element
// triangles + per-element buffer + per-DOF sums
double full_apply_bytes(const Level& lv, double wval, double wvec, bool r_minus) {
    const double nv = r_minus ? 3.0 : 2.0;
    if (!lv.eapply) return (double)lv.nnz * ((lv.sup ? lv.sup_ib : 4.0) + wval) + (double)lv.n * (8 + nv * wvec);
    const double nd = (double)lv.el.dofs.size();
    return (double)lv.etri_len * wval + nd * (4 + 8 + wvec + 2 * wval) + (double)lv.n * (8 + (nv - 1) * wvec);
}

// Finalize table of the large overlaps (launch_sub_finalize_tab): per sweep entry the
// scratch addresses of its partial sums for the level's chunk length.  Not built when
// the scratch exceeds int32 offsets (the finalize then looks the addresses up).
void build_fin_tab(lsdd_hierarchy* h, Level& lv, const std::vector<int64_t>& scr_off) {
    Arena& ar = h->arena;
    if (lv.d_fin_tab) {
        ar.release(lv.d_fin_tab);
        lv.d_fin_tab = nullptr;
    }
    const int32_t n_sub = (int32_t)lv.sw_sub_off.size() - 1;
    if (n_sub < 1 || scr_off[n_sub] >= (int64_t(1) << 31)) return;
    const int64_t rows = lv.sw_sub_off[n_sub];
    std::vector<int32_t> tab(4 * std::max<int64_t>(rows, 1), 0);
    for (int32_t q = 0; q < n_sub; ++q) {
        const int64_t o = lv.sw_sub_off[q], m = lv.sw_sub_off[q + 1] - o;
        if (m <= SMALL_M) continue;
        const int nt = (int)((m + 63) / 64);
        for (int64_t c = 0; c < m; ++c) {
            const int J = (int)(c >> 6), l = (int)(c & 63);
            int32_t* e = &tab[4 * (o + c)];
            e[0] = (int32_t)(scr_off[q] + symv_rowpart_off(J, lv.chl) * 64 + l);
            e[1] = (int32_t)(scr_off[q] + symv_rowpart_off(nt, lv.chl) * 64 + (int64_t)J * 64 + l);
            e[2] = J;
            e[3] = (J / lv.chl + 1) | (nt << 16);
        }
    }
    int32_t* d = ar.upload(tab, h->st);
    sync(h->st);
    if (reinterpret_cast<uintptr_t>(d) % 16 != 0) {   // a caller allocator without 16-byte alignment
        ar.release(d);
        return;
    }
    lv.d_fin_tab = d;
}

// Cycle vectors of one level: set b = 0 holds single vectors, b = 1 blocks of
// NRB interleaved right-hand sides.
void alloc_vectors(lsdd_hierarchy* h, Level& lv, int b) {
    Arena& a = h->arena;
    const int64_t w = b ? NRB : 1;
    const int64_t nl = std::max<int64_t>({lv.rloc_len, lv.c_dofs ? lv.term_len : 0, 1}) * w;
    const int64_t ns = std::max<int64_t>({lv.scr_len, lv.c_scr_len, 1}) * w;
    if (h->prm.precision >= 1) {
        VecSet<float>& v = lv.v32[b];
        v.r = a.alloc<float>(lv.n * w);
        v.x = a.alloc<float>(lv.n * w);
        v.t = a.alloc<float>(lv.n * w);
        v.rloc = a.alloc<float>(nl);
        v.scr = a.alloc<float>(ns);
        if (!lv.term.empty()) {
            lv.cr64[b] = a.alloc<double>(lv.n * w);
            lv.cx64[b] = a.alloc<double>(lv.n * w);
        }
    }
    VecSet<double>& v = lv.v64[b];
    v.r = a.alloc<double>(lv.n * w);
    v.x = a.alloc<double>(lv.n * w);
    v.t = a.alloc<double>(lv.n * w);
    v.rloc = a.alloc<double>(nl);
    v.scr = a.alloc<double>(ns);
}

template <class F>
void traced(lsdd_hierarchy* h, const char* name, double bytes, F&& launch) {
    if (!h->tr.on) {
        launch();
        return;
    }
    hipEvent_t a = h->tr.get(), b = h->tr.get();
    // the subdomain product takes the events into its launch (kernel start and end);
    // every other class is bracketed by event records on the stream
    const bool ext = !std::strcmp(name, "sub_symv") || !std::strcmp(name, "coarse_symv");
    if (ext) {
        set_launch_events(a, b);
        launch();
        hipEvent_t u, v;
        if (take_launch_events(&u, &v)) {     // nothing was launched: an empty interval
            HIPCHK(hipEventRecord(a, h->st));
            HIPCHK(hipEventRecord(b, h->st));
        }
    } else {
        HIPCHK(hipEventRecord(a, h->st));
        launch();
        HIPCHK(hipEventRecord(b, h->st));
    }
    h->tr.pend.push_back(Trace::Pend{h->tr.index(name), a, b, bytes});
}

// Work items (subdomain, tile row, chunk) of the symmetric subdomain kernel for
// the listed subdomains, longest chunks first (ties keep subdomain order).
void append_symv_items(const std::vector<int64_t>& sub_off, const std::vector<int32_t>& subs, int chl,
                       std::vector<int32_t>& items) {
    std::vector<int32_t> it;
    for (int32_t s : subs) sub_symv_items(s, sub_off[s + 1] - sub_off[s], chl, it);
    std::vector<size_t> ord(it.size() / 3);
    for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
    auto len = [&](size_t q) { return std::min(it[3 * q + 1] + 1 - chl * it[3 * q + 2], chl); };
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return len(a) > len(b); });
    for (size_t q : ord) items.insert(items.end(), {it[3 * q], it[3 * q + 1], it[3 * q + 2]});
}

// Terminal blocks of a level: the dense Cholesky factorisation and explicit
// inverse of the instance blocks of A_l listed in `term` (on the coarsest level:
// every instance present, i.e. the whole level for a single problem), packed into
// lower 64 x 64 tiles and applied by the symmetric subdomain kernel with one
// "subdomain" per block.
void make_terminal(lsdd_hierarchy* h, Level& lv, const std::vector<int32_t>& term, bool coarsest) {
    Arena& ar = h->arena;
    const int32_t nb = (int32_t)term.size();
    lv.term = term;
    std::vector<int64_t> sub_off(nb + 1, 0), inv_off(nb + 1, 0), tp_off(nb), scr_off(nb + 1, 0);
    std::vector<int32_t> dofs, pos;
    int64_t tiles = 0, max_ni = 0;
    lv.c_entries = 0.0;
    for (int32_t q = 0; q < nb; ++q) {
        const int64_t a = lv.inst_off[term[q]], ni = lv.inst_off[term[q] + 1] - a;
        max_ni = std::max(max_ni, ni);
        sub_off[q + 1] = sub_off[q] + ni;
        inv_off[q + 1] = inv_off[q] + ni * ni;
        tp_off[q] = tiles;
        const int64_t nt = (ni + 63) / 64;
        tiles += nt * (nt + 1) / 2 * 4096;
        scr_off[q + 1] = scr_off[q] + sub_symv_scratch_len(ni, lv.c_chl);
        lv.c_entries += (double)ni * (ni + 1) / 2.0;
        for (int64_t d = a; d < a + ni; ++d) {
            dofs.push_back((int32_t)d);
            pos.push_back(q);
        }
    }
    lv.term_len = sub_off[nb];
    bool identity = lv.term_len == lv.n;
    for (int64_t t = 0; identity && t < lv.term_len; ++t) identity = dofs[t] == t;
    if (max_ni > 49152) throw Error(LSDD_E_UNSUPPORTED, "terminal block too large: " + std::to_string(max_ni));
    // all blocks at once through the batched tiled engine: W <- chol(A_q),
    // X <- L^{-1} (forward solve on I), then A_q^{-1} = X^T X back into W
    double* W = ar.alloc<double>((size_t)inv_off[nb]);
    double* X = ar.alloc<double>((size_t)inv_off[nb]);
    double* d_minp = ar.alloc<double>(nb);
    double t0 = now_s();
    HIPCHK(hipMemsetAsync(W, 0, (size_t)inv_off[nb] * sizeof(double), h->st));
    std::vector<View> vq(nb);
    for (int32_t q = 0; q < nb; ++q) {
        const int64_t a = lv.inst_off[term[q]], ni = sub_off[q + 1] - sub_off[q];
        launch_dense_from_csr(a, ni, lv.d_rowptr, lv.d_col, lv.d_val, W + inv_off[q], h->st);
        vq[q] = View{inv_off[q], (int32_t)ni, (int32_t)ni, (int32_t)ni, 0};
    }
    Batched bt;
    bt.st = h->st;
    bt.alloc = [](void* c, size_t b) { return static_cast<Arena*>(c)->get(b); };
    bt.release = [](void* c, void* p) { static_cast<Arena*>(c)->release(p); };
    bt.ctx = &ar;
    bt.potrf(W, vq, d_minp);
    launch_views_identity(nb, X, bt.put(0, vq), h->st);
    bt.trsm(W, vq, X, vq, false, true);
    bt.gemm_tn(X, vq, X, vq, nullptr, vq, 0.0, W, vq, -1.0, true, true);
    std::vector<double> minp = download(d_minp, nb, h->st);
    bt.free_all();
    vlog("level %d: %d terminal block(s), %lld DOFs, dense Cholesky + inverse %.3f s", lv.level, nb,
         (long long)lv.term_len, now_s() - t0);
    ar.release(X);
    ar.release(d_minp);
    double* inv = W;
    for (int32_t q = 0; q < nb; ++q)
        if (!(minp[q] > 0.0))
            throw Error(LSDD_E_NUMERIC, "dense Cholesky of a terminal block failed (matrix not SPD), instance " +
                                            std::to_string(term[q]) + " on level " + std::to_string(lv.level));
    lv.c_sub_off = ar.upload(sub_off, h->st);
    lv.c_tp_off = ar.upload(tp_off, h->st);
    lv.c_scr_off = ar.upload(scr_off, h->st);
    lv.c_pos = ar.upload(pos, h->st);
    lv.c_dofs = identity ? nullptr : ar.upload(dofs, h->st);
    std::vector<int32_t> subs(nb), items;
    for (int32_t q = 0; q < nb; ++q) subs[q] = q;
    append_symv_items(sub_off, subs, lv.c_chl, items);
    lv.c_items = ar.upload(items, h->st);
    lv.c_nitems = (int64_t)items.size() / 3;
    lv.c_tiles = ar.alloc<double>(tiles);
    int64_t* d_inv_off = ar.upload(inv_off, h->st);
    launch_pack_tiles(nb, lv.c_sub_off, d_inv_off, inv, lv.c_tp_off, lv.c_tiles, nullptr, h->st);
    HIPCHK(hipGetLastError());
    sync(h->st);
    ar.release(d_inv_off);
    ar.release(inv);
    lv.c_scr_len = scr_off[nb];
    if (coarsest) {
        lv.coarsest = true;
        alloc_vectors(h, lv, 0);
    }
}

// Build level l+1 from level l; returns nullptr when no mode is retained.
std::unique_ptr<Level> coarsen(lsdd_hierarchy* h, Level& lv, const int32_t* agg_given) {
    const lsdd_params& P = h->prm;
    hipStream_t st = h->st;
    Arena& ar = h->arena;
    const int64_t n = lv.n;
    const double ta0 = now_s();
    // ---- aggregates
    int32_t n_agg = 0;
    if (agg_given) {
        lv.agg_of_dof.assign(agg_given, agg_given + n);
        n_agg = 1 + *std::max_element(lv.agg_of_dof.begin(), lv.agg_of_dof.end());
    } else {
        Csr g = supernode_graph(lv.n_super, lv.node_of_dof, lv.el);
        std::vector<int32_t> as = aggregate(g, lv.level == 0 ? P.agg_passes : P.agg_passes_coarse, &n_agg);
        lv.agg_of_dof.resize(n);
        for (int64_t d = 0; d < n; ++d) lv.agg_of_dof[d] = as[lv.node_of_dof[d]];
    }
    const int32_t n_inst = (int32_t)lv.inst_off.size() - 1;
    // instances whose hierarchy ends on this level take no part in aggregation
    if (!lv.term.empty()) {
        for (int32_t i : lv.term)
            for (int64_t d = lv.inst_off[i]; d < lv.inst_off[i + 1]; ++d) lv.agg_of_dof[d] = -1;
        std::vector<int32_t> newid(n_agg, -1);
        for (int64_t d = 0; d < n; ++d)
            if (lv.agg_of_dof[d] >= 0) newid[lv.agg_of_dof[d]] = 0;
        int32_t na = 0;
        for (int32_t a = 0; a < n_agg; ++a)
            if (newid[a] == 0) newid[a] = na++;
        for (int64_t d = 0; d < n; ++d)
            if (lv.agg_of_dof[d] >= 0) lv.agg_of_dof[d] = newid[lv.agg_of_dof[d]];
        n_agg = na;
    }
    // aggregates never span instances; number them instance-major (the order
    // inside an instance is kept), so every instance owns a contiguous range of
    // aggregates and hence of coarse DOFs
    std::vector<int32_t> inst_of_agg(n_agg, -1), agg_first(n_inst + 1, 0);
    {
        for (int32_t i = 0; i < n_inst; ++i)
            for (int64_t d = lv.inst_off[i]; d < lv.inst_off[i + 1]; ++d) {
                if (lv.agg_of_dof[d] < 0) continue;
                int32_t& ia = inst_of_agg[lv.agg_of_dof[d]];
                if (ia >= 0 && ia != i) throw Error(LSDD_E_INVAL, "an aggregate spans two instances");
                ia = i;
            }
        std::vector<int32_t> order(n_agg), newid(n_agg);
        for (int32_t a = 0; a < n_agg; ++a) order[a] = a;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return inst_of_agg[a] < inst_of_agg[b]; });
        std::vector<int32_t> ia2(n_agg);
        for (int32_t q = 0; q < n_agg; ++q) {
            newid[order[q]] = q;
            ia2[q] = inst_of_agg[order[q]];
        }
        for (int64_t d = 0; d < n; ++d)
            if (lv.agg_of_dof[d] >= 0) lv.agg_of_dof[d] = newid[lv.agg_of_dof[d]];
        inst_of_agg = ia2;
        for (int32_t a = 0; a < n_agg; ++a) agg_first[inst_of_agg[a] + 1]++;
        for (int32_t i = 0; i < n_inst; ++i) agg_first[i + 1] += agg_first[i];
    }
    lv.cl = build_closure(n, lv.agg_of_dof, n_agg, lv.el);
    if (P.closure == 1) {
        // algebraic A-closures from the numerical entries of A_l; the closure
        // elements and multiplicities stay those of the G-row closure, and the
        // local assembly drops element DOFs outside the smaller overlap
        const std::vector<double> val = download(lv.d_val, (size_t)lv.nnz, st);
        a_closure_overlaps(lv.pat, val, P.closure_tol, lv.cl);
    }
    const Closure& C = lv.cl;
    double tc0 = now_s();
    vlog("level %d: aggregation and closures %.3f s", lv.level, tc0 - ta0);
    for (int32_t i = 0; i < n_agg; ++i)
        if (C.agg_ptr[i + 1] == C.agg_ptr[i]) throw Error(LSDD_E_INVAL, "empty aggregate " + std::to_string(i));
    // smoother subdomains: the overlaps (multiplicative Schwarz, restricted additive
    // Schwarz) or the aggregates themselves (block Jacobi: disjoint, one class)
    const bool bj = P.smoother == 2;
    const std::vector<int64_t>& sp_ptr = bj ? C.agg_ptr : C.sub_ptr;
    const std::vector<int32_t>& sp_dofs = bj ? C.agg_dofs : C.sub_dofs;
    if (bj) {
        lv.colors.assign(n_agg, 0);
        lv.n_colors = n_agg > 0 ? 1 : 0;
    } else {
        lv.colors = color_subdomains(n, C, lv.el, &lv.n_colors);
    }
    vlog("level %d: colouring %.3f s", lv.level, now_s() - tc0);
    lv.smoother = P.smoother;
    const double tau_cut = P.tau_const * (double)C.max_mult;
    // tau_cut of every aggregate from the largest multiplicity of its own instance
    std::vector<double> thr_agg;
    if (n_inst > 1) {
        std::vector<int32_t> mm(n_inst, 0);
        for (int64_t e = 0; e < lv.el.count(); ++e) {
            const int32_t d = lv.el.dofs[lv.el.ptr[e]];
            const int32_t i = (int32_t)(std::upper_bound(lv.inst_off.begin(), lv.inst_off.end(), (int64_t)d) -
                                        lv.inst_off.begin() - 1);
            mm[i] = std::max(mm[i], C.mult[e]);
        }
        thr_agg.resize(n_agg);
        for (int32_t a = 0; a < n_agg; ++a) thr_agg[a] = 1.0 / (P.tau_const * (double)mm[inst_of_agg[a]]);
    }
    // ---- per-aggregate sizes and local positions of closure elements
    std::vector<int64_t> sq(n_agg + 1, 0), msq(n_agg + 1, 0);
    int64_t max_m = 0, max_nw = 0;
    for (int32_t i = 0; i < n_agg; ++i) {
        int64_t m = C.sub_ptr[i + 1] - C.sub_ptr[i], nw = C.agg_ptr[i + 1] - C.agg_ptr[i];
        max_m = std::max(max_m, m);
        max_nw = std::max(max_nw, nw);
        sq[i + 1] = sq[i] + nw * nw;
        msq[i + 1] = msq[i] + (bj ? nw * nw : m * m);   // smoother inverse
    }
    vlog("level %d: n=%lld aggregates=%d colours=%d max|omega|=%lld max|Omega|=%lld max mult=%d",
         lv.level, (long long)n, n_agg, lv.n_colors, (long long)max_nw, (long long)max_m, C.max_mult);
    if (max_m > 16384) throw Error(LSDD_E_UNSUPPORTED, "overlap larger than 16384 DOFs: " + std::to_string(max_m));
    if (max_nw > 4096) throw Error(LSDD_E_UNSUPPORTED, "aggregate larger than 4096 DOFs: " + std::to_string(max_nw));
    std::vector<int64_t> clpos_off(C.cl_elems.size() + 1, 0);
    std::vector<int32_t> clpos;
    {
        std::vector<int32_t> loc(n, -1);
        for (int32_t i = 0; i < n_agg; ++i) {
            for (int64_t q = C.sub_ptr[i]; q < C.sub_ptr[i + 1]; ++q) loc[C.sub_dofs[q]] = (int32_t)(q - C.sub_ptr[i]);
            for (int64_t c = C.cl_ptr[i]; c < C.cl_ptr[i + 1]; ++c) {
                int32_t e = C.cl_elems[c];
                for (int64_t r = lv.el.ptr[e]; r < lv.el.ptr[e + 1]; ++r) clpos.push_back(loc[lv.el.dofs[r]]);
                clpos_off[c + 1] = (int64_t)clpos.size();
            }
            for (int64_t q = C.sub_ptr[i]; q < C.sub_ptr[i + 1]; ++q) loc[C.sub_dofs[q]] = -1;
        }
    }
    vlog("level %d: closure positions %.3f s", lv.level, now_s() - tc0);
    // ---- device inputs
    int64_t* d_sub_ptr = ar.upload(C.sub_ptr, st);
    int32_t* d_sub_dofs = ar.upload(C.sub_dofs, st);
    lv.d_agg_ptr = ar.upload(C.agg_ptr, st);
    lv.d_agg_dofs = ar.upload(C.agg_dofs, st);
    int64_t* d_cl_ptr = ar.upload(C.cl_ptr, st);
    int32_t* d_cl_elems = ar.upload(C.cl_elems, st);
    int64_t* d_clpos_off = ar.upload(clpos_off, st);
    int32_t* d_clpos = ar.upload(clpos, st);
    int32_t* d_mult = ar.upload(C.mult, st);
    int64_t* d_inv_off = ar.upload(msq, st);
    int64_t* d_zst_off = ar.upload(sq, st);
    lv.inv_len = msq[n_agg];
    lv.d_inv = ar.alloc<double>(lv.inv_len);
    if (P.precision == 2) lv.d_X = ar.alloc<double>(lv.inv_len);
    double* d_zst = ar.alloc<double>(sq[n_agg]);
    lv.d_mu = ar.alloc<double>(n);
    lv.d_k = ar.alloc<int32_t>(n_agg);
    int32_t* d_status = ar.alloc<int32_t>(n_agg);
    HIPCHK(hipMemsetAsync(d_status, 0xff, n_agg * sizeof(int32_t), st));

    LocalArgs A{};
    A.sub_ptr = d_sub_ptr;
    A.sub_dofs = d_sub_dofs;
    A.agg_ptr = lv.d_agg_ptr;
    A.cl_ptr = d_cl_ptr;
    A.cl_elems = d_cl_elems;
    A.clpos_off = d_clpos_off;
    A.clpos = d_clpos;
    A.mult = d_mult;
    A.elem_ptr = lv.d_elem_ptr;
    A.blk_off = lv.d_blk_off;
    A.blocks = lv.d_blocks;
    A.rowptr = lv.d_rowptr;
    A.col = lv.d_col;
    A.val = lv.d_val;
    A.inv_off = d_inv_off;
    A.inv = lv.d_inv;
    A.zst_off = d_zst_off;
    A.zst = d_zst;
    A.mu_off = lv.d_agg_ptr;
    A.mu = lv.d_mu;
    A.k_out = lv.d_k;
    A.status = d_status;
    A.modes_fixed = P.modes_fixed;
    A.thr = 1.0 / tau_cut;
    double* d_thr = thr_agg.empty() ? nullptr : ar.upload(thr_agg, st);
    A.thr_agg = d_thr;
    A.band_tol = P.band_tol;
    A.trd_min = trd_min(P.blocked_eig_min);
    A.cluster_tol = P.cluster_tol;

    // ---- batched local problems (workspace bounded); every dense step runs as
    // tiled jobs of all aggregates of the batch at once
    // bytes of workspace per batch: half of the free device memory, at most 96 GiB and
    // at least 2 GiB.  The arithmetic of an aggregate does not depend on its batch;
    // larger batches share the per-column launches of the blocked eigensolver
    int64_t budget = int64_t(2) << 30;
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            budget = std::max<int64_t>(budget, std::min<int64_t>(int64_t(96) << 30, (int64_t)(free_b / 2)));
    }
    vlog("level %d: host graph work %.3f s", lv.level, now_s() - tc0);
    double tl0 = now_s();
    Batched bt;
    bt.st = st;
    bt.alloc = [](void* c, size_t b) { return static_cast<Arena*>(c)->get(b); };
    bt.release = [](void* c, void* p) { static_cast<Arena*>(c)->release(p); };
    bt.ctx = &ar;
    std::vector<int32_t> status(n_agg, 0);
    int32_t pos = 0;
    while (pos < n_agg) {
        std::vector<int64_t> ws_off(1, 0), sq_off(1, 0), t_off(1, 0);
        int32_t end = pos;
        int64_t bytes = 0;
        while (end < n_agg && (end - pos) < 32768) {
            int64_t m = C.sub_ptr[end + 1] - C.sub_ptr[end], nw = C.agg_ptr[end + 1] - C.agg_ptr[end];
            int64_t tl = 3 * nw + (int64_t)INVIT_SLOTS * nw + 4096;
            int64_t need = (2 * m * m + 2 * nw * nw + tl) * 8;
            if (end > pos && bytes + need > budget) break;
            bytes += need;
            ws_off.push_back(ws_off.back() + m * m);
            sq_off.push_back(sq_off.back() + nw * nw);
            t_off.push_back(t_off.back() + tl);
            ++end;
        }
        const int32_t nb = end - pos;
        double* w1 = ar.alloc<double>(ws_off.back());
        double* w2 = ar.alloc<double>(ws_off.back());
        double* sb = ar.alloc<double>(sq_off.back());
        double* vb = ar.alloc<double>(sq_off.back());
        double* tb = ar.alloc<double>(t_off.back());
        ws_off.pop_back();
        sq_off.pop_back();
        t_off.pop_back();
        int64_t* d_ws = ar.upload(ws_off, st);
        int64_t* d_sq = ar.upload(sq_off, st);
        int64_t* d_t = ar.upload(t_off, st);
        double* d_maxd = ar.alloc<double>(nb);
        double* d_minp = ar.alloc<double>(nb);
        LocalArgs B = A;
        B.first = pos;
        B.agg_list = nullptr;
        B.ws_off = d_ws;
        B.w1 = w1;
        B.w2 = w2;
        B.sq_off = d_sq;
        B.s_buf = sb;
        B.v_buf = vb;
        B.t_off = d_t;
        B.t_buf = tb;
        int32_t max_m = 0;
        for (int32_t b = 0; b < nb; ++b) max_m = std::max(max_m, (int32_t)(C.sub_ptr[pos + b + 1] - C.sub_ptr[pos + b]));
        launch_local_assemble(nb, B, max_m, st);
        std::vector<View> vGG, vGw, vww, vS, vAO, vLww;
        std::vector<int64_t> ngs(nb);
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t i = pos + b;
            const int32_t m = (int32_t)(C.sub_ptr[i + 1] - C.sub_ptr[i]), nw = (int32_t)(C.agg_ptr[i + 1] - C.agg_ptr[i]);
            const int32_t ng = m - nw;
            ngs[b] = ng;
            const int64_t o = ws_off[b];
            vGG.push_back(View{o + nw + (int64_t)nw * m, m, ng, ng, 0});
            vGw.push_back(View{o + nw, m, ng, nw, 0});
            vww.push_back(View{o, m, nw, nw, 0});
            vS.push_back(View{sq_off[b], nw, nw, nw, 0});
            vAO.push_back(View{o, m, m, m, 0});
            vLww.push_back(View{o, m, nw, nw, 0});
        }
        // Schur complement onto omega (eq. gep_reduced).  Cholesky of the interface
        // block; a block singular to working precision (a pivot <= |Gamma| eps max
        // diag) is assembled again and factored with diagonal pivoting, truncated when
        // the largest remaining diagonal entry falls to that tolerance: its Schur
        // complement is then taken over the eliminated (pivot) indices.  A~_Omega is
        // positive semidefinite, so the coupling lies in the range of the interface
        // block and this generalized inverse gives the Moore-Penrose Schur complement.
        HIPCHK(hipMemsetAsync(d_minp, 0x7f, nb * sizeof(double), st));
        launch_views_max_diag(nb, w1, bt.put(0, vGG), d_maxd, st);
        bt.potrf(w1, vGG, d_minp);
        {
            std::vector<double> maxd = download(d_maxd, nb, st), minp = download(d_minp, nb, st);
            std::vector<int32_t> sing, sing_b, lead;
            std::vector<int64_t> sing_ws;
            std::vector<double> tol;
            std::vector<View> vs;
            for (int32_t b = 0; b < nb; ++b) {
                if (ngs[b] == 0) continue;
                const double t = (double)ngs[b] * DBL_EPSILON * maxd[b];
                if (!(minp[b] > t)) {
                    sing.push_back(pos + b);
                    sing_b.push_back(b);
                    sing_ws.push_back(ws_off[b]);
                    tol.push_back(t);
                    vs.push_back(vAO[b]);
                    lead.push_back(vww[b].rows);
                }
            }
            if (!sing.empty()) {
                int32_t* d_list = ar.upload(sing, st);
                int64_t* d_sws = ar.upload(sing_ws, st);
                double* d_tol = ar.upload(tol, st);
                LocalArgs R = B;
                R.agg_list = d_list;
                R.ws_off = d_sws;
                int32_t sing_m = 0;
                for (int32_t i : sing) sing_m = std::max(sing_m, (int32_t)(C.sub_ptr[i + 1] - C.sub_ptr[i]));
                launch_local_assemble((int32_t)sing.size(), R, sing_m, st);
                std::vector<int32_t> rank;
                bt.pstrf_trailing(w1, vs, lead, d_tol, rank);
                int64_t dropped = 0;
                for (size_t t = 0; t < sing.size(); ++t) {
                    const int32_t b = sing_b[t];
                    vGG[b].rows = vGG[b].cols = rank[t];
                    vGw[b].rows = rank[t];
                    dropped += ngs[b] - rank[t];
                }
                vlog("  %zu interface blocks singular to working precision: pivoted, %lld indices dropped",
                     sing.size(), (long long)dropped);
                for (void* p : {(void*)d_list, (void*)d_sws, (void*)d_tol}) ar.release(p);
            }
        }
        bt.trsm(w1, vGG, w1, vGw, false);                                   // W = L_G^{-1} A~_Gw
        bt.gemm_tn(w1, vGw, w1, vGw, w1, vww, 1.0, sb, vS, 1.0);            // S~ = A~_ww - W^T W
        // Cholesky of A_Omega; its leading block is chol(A_ww)
        bt.potrf(w2, vAO, d_minp);
        {
            std::vector<double> minp = download(d_minp, nb, st);
            for (int32_t b = 0; b < nb; ++b)
                if (!(minp[b] > 0.0)) status[pos + b] = 2;
        }
        // C = L^{-1} S~ L^{-T}
        bt.trsm(w2, vLww, sb, vS, false);
        bt.transpose(sb, vS);
        bt.trsm(w2, vLww, sb, vS, false);
        launch_views_symmetrize(nb, sb, bt.put(0, vS), st);
        // eigenpairs of C and retained modes
        int32_t* d_big = nullptr;
        {
            int32_t mx = 0;
            std::vector<int32_t> big, bigsz;
            for (int32_t b = 0; b < nb; ++b) {
                const int32_t nw = (int32_t)(C.agg_ptr[pos + b + 1] - C.agg_ptr[pos + b]);
                mx = std::max(mx, nw);
                if (B.trd_min > 0 && nw >= B.trd_min) {
                    big.push_back(b);
                    bigsz.push_back(nw);
                }
            }
            if (!big.empty()) {
                d_big = ar.upload(big, st);
                launch_local_tridiag_blocked(B, d_big, bigsz, st);
            }
            launch_local_eig(nb, B, mx, 0, 1, st);
            if (!big.empty()) {
                // eigenvectors of the large problems: scratch sized by their mode counts
                std::vector<int32_t> ks(big.size());
                std::vector<int64_t> iw_off(big.size() + 1, 0);
                std::vector<int32_t> kall = download(lv.d_k + pos, nb, st);
                for (size_t t = 0; t < big.size(); ++t) {
                    ks[t] = kall[big[t]];
                    iw_off[t + 1] = iw_off[t] + (int64_t)((ks[t] + 63) / 64) * ((int64_t)INVIT_SLOTS * bigsz[t] + 4096);
                }
                double* iw = ar.alloc<double>(std::max<int64_t>(iw_off.back(), 1));
                int64_t* d_iw_off = ar.upload(iw_off, st);
                launch_local_invit_blocked(B, d_big, bigsz, ks, d_iw_off, iw, st);
                launch_local_eig(nb, B, mx, 2, 3, st);
                launch_local_backtransform_blocked(B, d_big, bigsz, st);
                sync(st);
                ar.release(iw);
                ar.release(d_iw_off);
            } else {
                launch_local_eig(nb, B, mx, 2, 3, st);
            }
        }
        HIPCHK(hipGetLastError());
        std::vector<int32_t> kb = download(lv.d_k + pos, nb, st);
        // Z = L_ww^{-T} V_k
        std::vector<View> vZ(nb);
        for (int32_t b = 0; b < nb; ++b) vZ[b] = View{ws_off[b], vS[b].rows, vS[b].rows, kb[b], 0};
        bt.trsm(w2, vLww, w1, vZ, true);
        launch_stage_z(nb, B, st);
        // smoother inverse A_Omega^{-1} = L^{-T} L^{-1}, or for block Jacobi
        // A_ww^{-1} from the leading block L_ww of the same factor
        {
            std::vector<View> vL(nb), vX(nb), vInv(nb);
            for (int32_t b = 0; b < nb; ++b) {
                const int32_t ms = bj ? vLww[b].rows : vAO[b].rows;
                vL[b] = bj ? vLww[b] : vAO[b];
                vX[b] = View{vAO[b].off, ms, ms, ms, 0};
                vInv[b] = View{msq[pos + b], ms, ms, ms, 0};
            }
            launch_views_identity(nb, w1, bt.put(0, vX), st);
            bt.trsm(w2, vL, w1, vX, false, true);                           // X = L^{-1} (lower)
            if (lv.d_X)
                for (int32_t b = 0; b < nb; ++b)
                    HIPCHK(hipMemcpyAsync(lv.d_X + msq[pos + b], w1 + vX[b].off,
                                          (size_t)vX[b].rows * vX[b].rows * sizeof(double), hipMemcpyDeviceToDevice,
                                          st));
            bt.gemm_tn(w1, vX, w1, vX, nullptr, vInv, 0.0, lv.d_inv, vInv, -1.0, true, true);   // X^T X
        }
        HIPCHK(hipGetLastError());
        sync(st);
        vlog("  batch of %d aggregates from %d done (%.3f s since start)", nb, pos, now_s() - tc0);
        bt.free_all();
        for (void* p : {(void*)w1, (void*)w2, (void*)sb, (void*)vb, (void*)tb, (void*)d_ws, (void*)d_sq, (void*)d_t,
                        (void*)d_maxd, (void*)d_minp})
            ar.release(p);
        if (d_big) ar.release(d_big);
        pos = end;
    }
    vlog("level %d: local problems %.3f s", lv.level, now_s() - tl0);
    const double tp0 = now_s();
    for (int32_t i = 0; i < n_agg; ++i) {
        if (status[i] != 0)
            throw Error(LSDD_E_NUMERIC, "local problem of aggregate " + std::to_string(i) +
                                            " failed (overlap matrix not SPD)");
    }
    lv.k = download(lv.d_k, n_agg, st);
    // ---- coarse numbering, compact Z
    lv.coff.assign(n_agg + 1, 0);
    lv.zoff.assign(n_agg + 1, 0);
    for (int32_t i = 0; i < n_agg; ++i) {
        lv.coff[i + 1] = lv.coff[i] + lv.k[i];
        lv.zoff[i + 1] = lv.zoff[i] + (C.agg_ptr[i + 1] - C.agg_ptr[i]) * lv.k[i];
    }
    lv.d_coff = ar.upload(lv.coff, st);
    lv.d_zoff = ar.upload(lv.zoff, st);
    lv.d_Z = ar.alloc<double>(lv.zoff[n_agg]);
    lv.d_Zc = ar.alloc<double>(lv.zoff[n_agg]);
    if (P.precision >= 1) lv.d_Zc32 = ar.alloc<float>(lv.zoff[n_agg]);
    launch_z_compact(n_agg, lv.d_agg_ptr, lv.d_k, d_zst_off, d_zst, lv.d_zoff, lv.d_Z, lv.d_Zc, lv.d_Zc32, st);
    {
        // aggregates up to SMALL_M DOFs: one thread per coarse DOF / entry; larger ones: work items
        std::vector<int32_t> ri, pi, aoc(std::max<int64_t>(lv.coff[n_agg], 1), -1),
            aop(std::max<int64_t>(C.agg_ptr[n_agg], 1), -1);
        for (int32_t i = 0; i < n_agg; ++i) {
            const int32_t nw = (int32_t)(C.agg_ptr[i + 1] - C.agg_ptr[i]);
            if (nw <= SMALL_M) {
                for (int64_t c = lv.coff[i]; c < lv.coff[i + 1]; ++c) aoc[c] = i;
                if (lv.k[i] > 0)
                    for (int64_t q = C.agg_ptr[i]; q < C.agg_ptr[i + 1]; ++q) aop[q] = i;
                continue;
            }
            for (int32_t s0 = 0; s0 < lv.k[i]; s0 += 16) { ri.push_back(i); ri.push_back(s0); }
            if (lv.k[i] > 0)
                for (int32_t r0 = 0; r0 < nw; r0 += 256) { pi.push_back(i); pi.push_back(r0); }
        }
        lv.n_ritems = (int64_t)ri.size() / 2;
        lv.n_pitems = (int64_t)pi.size() / 2;
        lv.d_ritems = ar.upload(ri, st);
        lv.d_pitems = ar.upload(pi, st);
        lv.d_agg_of_c = ar.upload(aoc, st);
        lv.d_agg_of_p = ar.upload(aop, st);
        lv.n_aggent = C.agg_ptr[n_agg];
    }
    sync(st);
    ar.release(d_zst);
    // ---- smoother arrays in sweep order: colour-major; inside a colour the large
    // overlaps (tiled product) come first, then the small ones (|Omega| <= SMALL_M);
    // subdomains of one colour commute, so this order gives the same smoother
    auto is_small = [&](int32_t i) { return sp_ptr[i + 1] - sp_ptr[i] <= SMALL_M; };
    lv.sweep.resize(n_agg);
    for (int32_t i = 0; i < n_agg; ++i) lv.sweep[i] = i;
    std::stable_sort(lv.sweep.begin(), lv.sweep.end(), [&](int32_t a, int32_t b) {
        if (lv.colors[a] != lv.colors[b]) return lv.colors[a] < lv.colors[b];
        return (int)is_small(a) < (int)is_small(b);
    });
    std::vector<int32_t> sw_dofs, sw_dofs_w;
    std::vector<int64_t> tp_agg(n_agg, -1), pk_agg(n_agg, -1), sw_tp_off(n_agg, -1), sw_pk_off(n_agg, -1);
    int64_t tiles = 0, pks = 0;
    for (int32_t i = 0; i < n_agg; ++i) {
        const int64_t m = sp_ptr[i + 1] - sp_ptr[i];
        if (is_small(i)) {
            pk_agg[i] = pks;
            pks += m * (m + 1) / 2;
        } else {
            const int64_t nt = (m + 63) / 64;
            tp_agg[i] = tiles;
            tiles += nt * (nt + 1) / 2 * 4096;
        }
    }
    lv.tiles_len = tiles;
    std::vector<int32_t> items;
    lv.sw_sub_off.assign(1, 0);
    lv.color_row0.assign(lv.n_colors + 1, 0);
    lv.color_rmid.assign(lv.n_colors, 0);
    lv.color_sub0.assign(lv.n_colors + 1, 0);
    lv.color_smid.assign(lv.n_colors, 0);
    lv.color_item0.assign(lv.n_colors + 1, 0);
    for (int32_t c = 0; c < lv.n_colors; ++c) lv.color_smid[c] = -1;
    for (int32_t s = 0; s < n_agg; ++s) {
        int32_t i = lv.sweep[s];
        int32_t c = lv.colors[i];
        if (is_small(i) && lv.color_smid[c] < 0) {
            lv.color_smid[c] = s;
            lv.color_rmid[c] = (int64_t)sw_dofs.size();
        }
        if (is_small(i)) lv.small_m = std::max<int32_t>(lv.small_m, (int32_t)(sp_ptr[i + 1] - sp_ptr[i]));
        sw_dofs.insert(sw_dofs.end(), sp_dofs.begin() + sp_ptr[i], sp_dofs.begin() + sp_ptr[i + 1]);
        // the same list with the interface entries masked (-1): the aggregate part
        // of the overlap, for the restricted updates of RAS
        const int64_t nw_i = C.agg_ptr[i + 1] - C.agg_ptr[i];
        for (int64_t q = sp_ptr[i]; q < sp_ptr[i + 1]; ++q) sw_dofs_w.push_back(q - sp_ptr[i] < nw_i ? sp_dofs[q] : -1);
        lv.sw_sub_off.push_back((int64_t)sw_dofs.size());
        sw_tp_off[s] = tp_agg[i];
        sw_pk_off[s] = pk_agg[i];
        lv.color_row0[c + 1] = (int64_t)sw_dofs.size();
        lv.color_sub0[c + 1] = s + 1;
    }
    for (int32_t c = 0; c < lv.n_colors; ++c)
        if (lv.color_smid[c] < 0) {            // no small overlap in this colour
            lv.color_smid[c] = lv.color_sub0[c + 1];
            lv.color_rmid[c] = lv.color_row0[c + 1];
        }
    // work items of the large overlaps per colour: (subdomain, tile row, chunk), longest chunks first
    for (int32_t c = 0; c < lv.n_colors; ++c) {
        std::vector<int32_t> subs;
        for (int32_t s = lv.color_sub0[c]; s < lv.color_smid[c]; ++s) subs.push_back(s);
        append_symv_items(lv.sw_sub_off, subs, lv.chl, items);
        lv.color_item0[c + 1] = (int64_t)items.size() / 3;
    }
    lv.color_m2.assign(lv.n_colors, 0.0);
    lv.color_m.assign(lv.n_colors, 0.0);
    lv.color_nnz.assign(lv.n_colors, 0.0);
    lv.color_pk.assign(lv.n_colors, 0.0);
    for (int32_t i = 0; i < n_agg; ++i) {
        double m = (double)(sp_ptr[i + 1] - sp_ptr[i]);
        (is_small(i) ? lv.color_pk : lv.color_m2)[lv.colors[i]] += m * (m + 1.0) / 2.0;   // inverse entries
        lv.color_m[lv.colors[i]] += m;
        for (int64_t q = sp_ptr[i]; q < sp_ptr[i + 1]; ++q) {
            int32_t d = sp_dofs[q];
            lv.color_nnz[lv.colors[i]] += (double)(lv.pat.ptr[d + 1] - lv.pat.ptr[d]);
        }
    }
    for (int32_t c = 0; c < lv.n_colors; ++c)
        vlog("  colour %d: %lld DOFs, %lld items, %.1f MB of inverse tiles; %d small overlaps, %.1f MB packed", c,
             (long long)(lv.color_row0[c + 1] - lv.color_row0[c]),
             (long long)(lv.color_item0[c + 1] - lv.color_item0[c]), lv.color_m2[c] * 8e-6,
             lv.color_sub0[c + 1] - lv.color_smid[c], lv.color_pk[c] * 8e-6);
    lv.d_sw_sub_off = ar.upload(lv.sw_sub_off, st);
    lv.d_sw_sub_dofs = ar.upload(sw_dofs, st);
    if (lv.d_scoff && (int64_t)lv.node_of_dof.size() == lv.n && sw_dofs.size() < (size_t)INT32_MAX) {
        // supernode row blocks of the sweep list: runs of up to 8 entries of one
        // colour whose rows belong to one supernode (so share one column list)
        std::vector<int32_t> rb;
        lv.color_rblk0.assign(lv.n_colors + 1, 0);
        for (int32_t c = 0; c < lv.n_colors; ++c) {
            const int64_t t1 = lv.color_row0[c + 1];
            for (int64_t t = lv.color_row0[c]; t < t1;) {
                const int32_t sn = lv.node_of_dof[sw_dofs[t]];
                int64_t e = t + 1;
                while (e < t1 && e - t < 8 && lv.node_of_dof[sw_dofs[e]] == sn) ++e;
                rb.push_back((int32_t)t);
                rb.push_back((int32_t)(e - t));
                t = e;
            }
            lv.color_rblk0[c + 1] = (int64_t)rb.size() / 2;
        }
        lv.d_rblk = ar.upload(rb, st);
    }
    if (P.smoother == 1) lv.d_sw_sub_dofs_w = ar.upload(sw_dofs_w, st);
    lv.d_sw_tp_off = ar.upload(sw_tp_off, st);
    lv.d_items = ar.upload(items, st);
    if (P.precision == 2) {
        // whole-tile-row items of the one-pass factor product, longest rows first per colour
        std::vector<int32_t> ritems;
        lv.color_ritem0.assign(lv.n_colors + 1, 0);
        lv.color_stash.assign(lv.n_colors, 0);
        for (int32_t c = 0; c < lv.n_colors; ++c) {
            std::vector<std::pair<int32_t, int32_t>> rows;
            for (int32_t q = lv.color_sub0[c]; q < lv.color_smid[c]; ++q) {
                const int32_t nt = (int32_t)((lv.sw_sub_off[q + 1] - lv.sw_sub_off[q] + 63) / 64);
                for (int32_t I = 0; I < nt; ++I) rows.emplace_back(q, I);
            }
            std::stable_sort(rows.begin(), rows.end(),
                             [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                                 return a.second > b.second;
                             });
            for (auto& r : rows) ritems.insert(ritems.end(), {r.first, r.second});
            lv.color_ritem0[c + 1] = (int64_t)ritems.size() / 2;
            // the longest tile row of the colour, up to the LDS capacity
            lv.color_stash[c] = rows.empty() ? 0 : std::min<int>(SUB_FACT_MAX_STASH, rows.front().second + 1);
        }
        lv.d_row_items = ar.upload(ritems, st);
    }
    {
        std::vector<int32_t> pos_sub(sw_dofs.size());
        std::vector<int64_t> scr_off(n_agg + 1, 0);
        for (int32_t s = 0; s < n_agg; ++s) {
            for (int64_t q = lv.sw_sub_off[s]; q < lv.sw_sub_off[s + 1]; ++q) pos_sub[q] = s;
            const int64_t m = lv.sw_sub_off[s + 1] - lv.sw_sub_off[s];
            scr_off[s + 1] = scr_off[s] + (m <= SMALL_M ? 0 : sub_symv_scratch_len(m, lv.chl));
        }
        lv.d_pos_sub = ar.upload(pos_sub, st);
        lv.d_scr_off = ar.upload(scr_off, st);
        lv.scr_len = scr_off[n_agg];
        build_fin_tab(h, lv, scr_off);
        lv.color_scr.assign(lv.n_colors, 0.0);
        for (int32_t q = 0; q < n_agg; ++q) lv.color_scr[lv.colors[lv.sweep[q]]] += (double)(scr_off[q + 1] - scr_off[q]);
    }
    {
        int64_t* d_tp_agg = ar.upload(tp_agg, st);
        int64_t* d_pk_agg = ar.upload(pk_agg, st);
        lv.d_sw_pk_off = ar.upload(sw_pk_off, st);
        lv.d_tiles = ar.alloc<double>(std::max<int64_t>(lv.tiles_len, 1));
        if (P.precision >= 1) lv.d_tiles32 = ar.alloc<float>(std::max<int64_t>(lv.tiles_len, 1));
        lv.d_pk = ar.alloc<double>(std::max<int64_t>(pks, 1));
        if (P.precision >= 1) lv.d_pk32 = ar.alloc<float>(std::max<int64_t>(pks, 1));
        const int64_t* d_sp_ptr = bj ? lv.d_agg_ptr : d_sub_ptr;
        launch_pack_tiles(n_agg, d_sp_ptr, d_inv_off, lv.d_inv, d_tp_agg, lv.d_tiles, lv.d_tiles32, st);
        launch_pack_small(n_agg, d_sp_ptr, d_inv_off, lv.d_inv, d_pk_agg, lv.d_pk, lv.d_pk32, st);
        if (lv.d_X) {
            // the factors X = L^{-1} in the same storage, FP32 only
            lv.d_tfac32 = ar.alloc<float>(std::max<int64_t>(lv.tiles_len, 1));
            lv.d_pkfac32 = ar.alloc<float>(std::max<int64_t>(pks, 1));
            launch_pack_tiles(n_agg, d_sp_ptr, d_inv_off, lv.d_X, d_tp_agg, nullptr, lv.d_tfac32, st);
            launch_pack_small(n_agg, d_sp_ptr, d_inv_off, lv.d_X, d_pk_agg, nullptr, lv.d_pkfac32, st);
        }
        HIPCHK(hipGetLastError());
        sync(st);
        if (lv.d_X) {
            ar.release(lv.d_X);
            lv.d_X = nullptr;
        }
        ar.release(d_tp_agg);
        ar.release(d_pk_agg);
        ar.release(lv.d_inv);
        lv.d_inv = nullptr;
    }
    lv.rloc_len = (int64_t)sw_dofs.size();
    alloc_vectors(h, lv, 0);
    // free local-problem inputs that the solve does not use
    for (void* p : {(void*)d_sub_ptr, (void*)d_sub_dofs, (void*)d_cl_ptr, (void*)d_cl_elems, (void*)d_clpos_off,
                    (void*)d_clpos, (void*)d_mult, (void*)d_inv_off, (void*)d_zst_off, (void*)d_status})
        ar.release(p);
    if (d_thr) ar.release(d_thr);
    const int64_t nc = lv.coff[n_agg];
    // coarse DOF ranges of the instances; an instance without retained modes
    // would end its hierarchy here while the others continue
    std::vector<int64_t> c_inst_off(n_inst + 1);
    int32_t n_empty = 0;
    for (int32_t i = 0; i <= n_inst; ++i) c_inst_off[i] = lv.coff[agg_first[i]];
    for (int32_t i = 0; i < n_inst; ++i)
        n_empty += agg_first[i + 1] > agg_first[i] && c_inst_off[i + 1] == c_inst_off[i];
    if (nc == 0) return nullptr;
    if (n_empty > 0)
        throw Error(LSDD_E_UNSUPPORTED, "an instance of the batch retains no mode on level " +
                                            std::to_string(lv.level) + " while others do");
    vlog("level %d: modes, transfers, sweep order and packed inverses %.3f s", lv.level, now_s() - tp0);
    // ---- coarse level: grouped element rows and Galerkin products
    const double tg00 = now_s();
    CoarseGroups G = group_coarse(lv.el, lv.agg_of_dof, lv.k, lv.coff);
    auto cv = std::make_unique<Level>();
    cv->level = lv.level + 1;
    cv->n = nc;
    cv->inst_off = c_inst_off;
    cv->el = std::move(G.coarse);
    cv->node_of_dof = G.node_of_cdof;
    cv->n_super = G.n_super;
    const int64_t ng = cv->el.count();
    cv->blk_off.assign(ng + 1, 0);
    std::vector<int64_t> pm_off(G.mem_elems.size() + 1, 0), pm_zrow;
    std::vector<int32_t> pm_k, pm_col;
    pm_zrow.reserve(lv.el.dofs.size());
    pm_k.reserve(lv.el.dofs.size());
    pm_col.reserve(lv.el.dofs.size());
    std::vector<int32_t> colof(n_agg, -1), agg_of_c(nc);
    for (int32_t a = 0; a < n_agg; ++a)
        for (int64_t d = lv.coff[a]; d < lv.coff[a + 1]; ++d) agg_of_c[d] = a;
    std::vector<int32_t> touched;
    for (int64_t g = 0; g < ng; ++g) {
        int64_t c = cv->el.ptr[g + 1] - cv->el.ptr[g];
        cv->blk_off[g + 1] = cv->blk_off[g] + c * c;
        // column offset of each aggregate inside the group support
        int64_t off = 0;
        touched.clear();
        for (int64_t q = cv->el.ptr[g]; q < cv->el.ptr[g + 1];) {
            int32_t d = cv->el.dofs[q];
            int32_t agg = agg_of_c[d];
            colof[agg] = (int32_t)off;
            touched.push_back(agg);
            off += lv.k[agg];
            q += lv.k[agg];
        }
        for (int64_t mi = G.mem_ptr[g]; mi < G.mem_ptr[g + 1]; ++mi) {
            int32_t e = G.mem_elems[mi];
            for (int64_t r = lv.el.ptr[e]; r < lv.el.ptr[e + 1]; ++r) {
                int32_t d = lv.el.dofs[r];
                int32_t agg = lv.agg_of_dof[d];
                if (lv.k[agg] > 0) {
                    pm_zrow.push_back(lv.zoff[agg] + (int64_t)C.pos_in_agg[d] * lv.k[agg]);
                    pm_k.push_back(lv.k[agg]);
                    pm_col.push_back(colof[agg]);
                } else {
                    pm_zrow.push_back(-1);
                    pm_k.push_back(0);
                    pm_col.push_back(0);
                }
            }
            pm_off[mi + 1] = (int64_t)pm_zrow.size();
        }
        for (int32_t agg : touched) colof[agg] = -1;
    }
    upload_elements(h, *cv);
    cv->d_blocks = ar.alloc<double>(cv->blk_off[ng]);
    double tg0 = now_s();
    {
        // stacked interpolation rows P_g per group, Y_e = F_e P_e per member,
        // then A_g = Y^T Y (Gram factors) or P_g^T Y, both on the matrix cores
        const bool gram = lv.level == 0;
        const bool g32 = h->prm.galerkin_precision == 1;
        const double* fb = gram ? lv.d_G : lv.d_blocks;
        std::vector<int64_t> R(ng, 0);
        for (int64_t g = 0; g < ng; ++g)
            for (int64_t mi = G.mem_ptr[g]; mi < G.mem_ptr[g + 1]; ++mi) {
                const int32_t e = G.mem_elems[mi];
                R[g] += lv.el.ptr[e + 1] - lv.el.ptr[e];
            }
        PstArgs pa{};
        pa.cptr = cv->d_elem_ptr;
        pa.mem_ptr = ar.upload(G.mem_ptr, st);
        pa.mem_elems = ar.upload(G.mem_elems, st);
        pa.felem_ptr = lv.d_elem_ptr;
        pa.pm_off = ar.upload(pm_off, st);
        pa.pm_zrow = ar.upload(pm_zrow, st);
        pa.pm_k = ar.upload(pm_k, st);
        pa.pm_col = ar.upload(pm_col, st);
        pa.Z = lv.d_Z;
        Batched bt;
        bt.st = st;
        bt.alloc = [](void* c, size_t b) { return static_cast<Arena*>(c)->get(b); };
        bt.release = [](void* c, void* p) { static_cast<Arena*>(c)->release(p); };
        bt.ctx = &ar;
        const int64_t budget = int64_t(2) << 30;    // bytes of P and Y per launch batch
        constexpr size_t MAXV = 65535;              // views per launch
        int64_t g0 = 0;
        while (g0 < ng) {
            int64_t g1 = g0, tot = 0;
            std::vector<int64_t> off, rows;
            while (g1 < ng) {
                const int64_t c = cv->el.ptr[g1 + 1] - cv->el.ptr[g1], sz = R[g1] * c;
                if (g1 > g0 && (tot + sz) * 16 > budget) break;
                off.push_back(tot);
                rows.push_back(R[g1]);
                tot += sz;
                ++g1;
            }
            double* pst = ar.alloc<double>(std::max<int64_t>(tot, 1));
            double* y = ar.alloc<double>(std::max<int64_t>(tot, 1));
            pa.g0 = (int32_t)g0;
            pa.n_groups = (int32_t)(g1 - g0);
            pa.pst_off = ar.upload(off, st);
            pa.rows = ar.upload(rows, st);
            pa.pst = pst;
            launch_build_pst(pa, st);
            std::vector<View> va, vb;
            auto flush_members = [&]() {
                if (va.empty()) return;
                bt.gemm_tn(fb, va, pst, vb, nullptr, vb, 0.0, y, vb, -1.0, false, false, g32);
                va.clear();
                vb.clear();
            };
            for (int64_t g = g0; g < g1; ++g) {
                const int32_t c = (int32_t)(cv->el.ptr[g + 1] - cv->el.ptr[g]);
                int64_t r0 = 0;
                for (int64_t mi = G.mem_ptr[g]; mi < G.mem_ptr[g + 1]; ++mi) {
                    const int32_t e = G.mem_elems[mi];
                    const int32_t ne = (int32_t)(lv.el.ptr[e + 1] - lv.el.ptr[e]);
                    va.push_back(View{lv.blk_off[e], ne, ne, ne, 0});
                    vb.push_back(View{off[g - g0] + r0, (int32_t)R[g], ne, c, 0});
                    r0 += ne;
                    if (va.size() == MAXV) flush_members();
                }
            }
            flush_members();
            std::vector<View> wa, wc;
            auto flush_groups = [&]() {
                if (wa.empty()) return;
                bt.gemm_tn(gram ? y : pst, wa, y, wa, nullptr, wc, 0.0, cv->d_blocks, wc, -1.0, false, true, g32);
                wa.clear();
                wc.clear();
            };
            for (int64_t g = g0; g < g1; ++g) {
                const int32_t c = (int32_t)(cv->el.ptr[g + 1] - cv->el.ptr[g]);
                wa.push_back(View{off[g - g0], (int32_t)R[g], (int32_t)R[g], c, 0});
                wc.push_back(View{cv->blk_off[g], c, c, c, 0});
                if (wa.size() == MAXV) flush_groups();
            }
            flush_groups();
            HIPCHK(hipGetLastError());
            sync(st);
            for (const void* p : {(const void*)pst, (const void*)y, (const void*)pa.pst_off, (const void*)pa.rows})
                ar.release(const_cast<void*>(p));
            g0 = g1;
        }
        bt.free_all();
        for (const void* p : {(const void*)pa.mem_ptr, (const void*)pa.mem_elems, (const void*)pa.pm_off,
                              (const void*)pa.pm_zrow, (const void*)pa.pm_k, (const void*)pa.pm_col})
            ar.release(const_cast<void*>(p));
    }
    vlog("level %d: Galerkin products for %lld coarse elements %.3f s (grouping %.3f s)", lv.level, (long long)ng,
         now_s() - tg0, tg0 - tg00);
    const double tas = now_s();
    assemble_operator(h, *cv);
    sync(st);
    vlog("level %d: coarse operator assembly %.3f s", cv->level, now_s() - tas);
    return cv;
}

// ---------------------------------------------------------------- V-cycle

template <typename T>
struct LvOps;
template <>
struct LvOps<double> {
    static VecSet<double>& v(Level& l, int b) { return l.v64[b]; }
    static const double* val(Level& l) { return l.d_val; }
    static const double* Z(Level& l) { return l.d_Zc; }
    static const double* inv(Level& l) { return l.d_tiles; }
    static const double* pk(Level& l) { return l.d_pk; }
    static const double* etri(Level& l) { return l.d_etri; }
    static double* ebuf(Level& l) { return l.d_ebuf; }
};
template <>
struct LvOps<float> {
    static VecSet<float>& v(Level& l, int b) { return l.v32[b]; }
    static const float* val(Level& l) { return l.d_val32; }
    static const float* Z(Level& l) { return l.d_Zc32; }
    static const float* inv(Level& l) { return l.d_tiles32; }
    static const float* pk(Level& l) { return l.d_pk32; }
    static const float* etri(Level& l) { return l.d_etri32; }
    static float* ebuf(Level& l) { return l.d_ebuf32; }
};

// Cycle kernels for NR = 1 (single vectors) or NR = NRB (interleaved blocks).
template <typename T, int NR>
struct Cyc {
    static void resid_rows(int64_t nrows, const int32_t* rows, Level& lv, const T* val, const T* x, const T* r, T* out,
                           bool xz, hipStream_t st) {
        if constexpr (NR == 1)
            launch_csr_resid_rows<T>(nrows, rows, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col, val, x, r, out, xz,
                                     lv.lanes, st, lv.sup ? lv.d_scoff : nullptr);
        else
            launch_csr_resid_rows_b<T>(nrows, rows, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col, val, x, r, out, xz,
                                       lv.lanes_b, st, lv.sup ? lv.d_scoff : nullptr);
    }
    // the residual rows of colour c of a sweep into rloc (indexed like the whole
    // sweep list), values of type V; by supernode row blocks where chosen
    template <typename V>
    static void resid_colour(Level& lv, int32_t c, const V* val, const T* x, const T* r, T* rloc, bool xz,
                             hipStream_t st) {
        const int64_t r0 = lv.color_row0[c], r1 = lv.color_row0[c + 1];
        if constexpr (NR == 1) {
            if (lv.sup >= 2 && lv.d_rblk) {
                const int64_t b0 = lv.color_rblk0[c];
                launch_sup_resid_blocks<T, V>(lv.color_rblk0[c + 1] - b0, lv.d_rblk + 2 * b0, lv.d_sw_sub_dofs,
                                              lv.d_rowptr, lv.d_scol, lv.d_scoff, val, x, r, rloc, xz,
                                              1 << (lv.sup - 2), st);
                return;
            }
            launch_csr_resid_rows<T, V>(r1 - r0, lv.d_sw_sub_dofs + r0, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col,
                                        val, x, r, rloc + r0, xz, lv.lanes, st, lv.sup ? lv.d_scoff : nullptr);
        } else {
            if (lv.sup >= 2 && lv.d_rblk && lv.lanes_b <= 16) {
                const int64_t b0 = lv.color_rblk0[c];
                launch_sup_resid_blocks_b<T>(lv.color_rblk0[c + 1] - b0, lv.d_rblk + 2 * b0, lv.d_sw_sub_dofs,
                                             lv.d_rowptr, lv.d_scol, lv.d_scoff, val, x, r, rloc, xz, lv.lanes_b, st);
                return;
            }
            resid_rows(r1 - r0, lv.d_sw_sub_dofs + r0, lv, val, x, r, rloc + r0 * NR, xz, st);
        }
    }
    // y = A x or r_minus - A x with the level's entries of type T (val), or from its
    // element triangles of the same precision when the autotuner chose them
    static void spmv(Level& lv, const T* val, const T* x, T* y, const T* r_minus, hipStream_t st) {
        if constexpr (NR == 1) {
            if (lv.eapply && LvOps<T>::etri(lv)) {
                launch_elem_apply<T, T>(lv.el.count(), lv.d_elem_ptr, lv.d_elem_dofs, lv.d_etri_off, LvOps<T>::etri(lv),
                                        lv.e_nmax, x, LvOps<T>::ebuf(lv), lv.n, lv.d_d2e_ptr, lv.d_e2y, r_minus, y, st);
                return;
            }
            launch_csr_spmv<T>(lv.n, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col, val, x, y, r_minus, lv.lanes, st,
                               lv.sup ? lv.d_scoff : nullptr);
        } else {
            launch_csr_spmv_b<T>(lv.n, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col, val, x, y, r_minus, lv.lanes_b, st,
                                 lv.sup ? lv.d_scoff : nullptr);
        }
    }
    static void symv(int64_t n_items, const int32_t* items, const int64_t* sub_off, const int64_t* tp_off,
                     const T* tiles, const T* rloc, const int64_t* scr_off, T* scr, int chl, hipStream_t st) {
        if constexpr (NR == 1) launch_sub_symv<T>(n_items, items, sub_off, tp_off, tiles, rloc, scr_off, scr, chl, st);
        else launch_sub_symv_b<T>(n_items, items, sub_off, tp_off, tiles, rloc, scr_off, scr, chl, st);
    }
    static void finalize(int64_t r0, int64_t r1, const int32_t* pos, const int64_t* sub_off, const int64_t* scr_off,
                         const T* scr, const int32_t* dofs, T* x, bool acc, int chl, int fl, hipStream_t st) {
        if constexpr (NR == 1) launch_sub_finalize<T>(r0, r1, pos, sub_off, scr_off, scr, dofs, x, acc, chl, fl, st);
        else launch_sub_finalize_b<T>(r0, r1, pos, sub_off, scr_off, scr, dofs, x, acc, chl, fl, st);
    }
    // x += the large-overlap corrections of colour c of a sweep (scatter list dofs)
    static void finalize_colour(Level& lv, int32_t c, const T* scr, const int32_t* dofs, T* x, hipStream_t st) {
        const int64_t r0 = lv.color_row0[c], rm = lv.color_rmid[c];
        if (lv.d_fin_tab && dofs) {
            if constexpr (NR == 1) launch_sub_finalize_tab<T>(r0, rm, lv.d_fin_tab, scr, dofs, x, lv.fl, st);
            else launch_sub_finalize_tab_b<T>(r0, rm, lv.d_fin_tab, scr, dofs, x, lv.fl, st);
            return;
        }
        finalize(r0, rm, lv.d_pos_sub, lv.d_sw_sub_off, lv.d_scr_off, scr, dofs, x, true, lv.chl, lv.fl, st);
    }
    static void small(Level& lv, int64_t s0, int64_t n_sub, const T* pk, const T* rloc, T* x, const int32_t* dofs,
                      hipStream_t st) {
        launch_small_sub<T, NR>(s0, n_sub, lv.d_sw_sub_off, dofs, lv.d_sw_pk_off, pk, rloc, x, lv.small_m, st);
    }
    static void restrict_(Level& lv, const T* Z, const T* t, T* rc, hipStream_t st) {
        launch_restrict_small<T, NR>(lv.coff.back(), lv.d_agg_of_c, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_coff,
                                     Z, t, rc, st);
        if constexpr (NR == 1)
            launch_restrict<T>(lv.n_ritems, lv.d_ritems, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_k, lv.d_coff, Z,
                               t, rc, st);
        else
            launch_restrict_b<T>(lv.n_ritems, lv.d_ritems, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_k, lv.d_coff,
                                 Z, t, rc, st);
    }
    static void prolong(Level& lv, const T* Z, const T* ec, T* x, hipStream_t st) {
        launch_prolong_small<T, NR>(lv.n_aggent, lv.d_agg_of_p, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_k,
                                    lv.d_coff, Z, ec, x, st);
        if constexpr (NR == 1)
            launch_prolong<T>(lv.n_pitems, lv.d_pitems, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_k, lv.d_coff, Z,
                              ec, x, st);
        else
            launch_prolong_b<T>(lv.n_pitems, lv.d_pitems, lv.d_agg_ptr, lv.d_agg_dofs, lv.d_zoff, lv.d_k, lv.d_coff,
                                Z, ec, x, st);
    }
};

// Restricted additive Schwarz step (Sec. 2, block Schwarz smoothers): all local
// residuals from the same x, then the local solves.  Pre-smoother M^{-1}: full
// local residuals, corrections kept on the aggregates (interface entries of the
// scatter list masked); post-smoother M^{-T}: residuals restricted to the
// aggregates (masked gather), full corrections.  The corrections of one colour
// are disjoint, so the colours are applied one after the other.
template <typename T, int NR>
void sweep_ras(lsdd_hierarchy* h, Level& lv, const T* r, T* x, bool post, bool x_zero_first) {
    using O = LvOps<T>;
    using C = Cyc<T, NR>;
    VecSet<T>& v = O::v(lv, NR > 1);
    const double w = (double)sizeof(T), wv = w * NR;
    const int64_t rows = lv.color_row0[lv.n_colors];
    double m_all = 0.0, nnz_all = 0.0;
    for (int32_t c = 0; c < lv.n_colors; ++c) {
        m_all += lv.color_m[c];
        nnz_all += lv.color_nnz[c];
    }
    const int32_t* gather = post ? lv.d_sw_sub_dofs_w : lv.d_sw_sub_dofs;
    const int32_t* scatter = post ? lv.d_sw_sub_dofs : lv.d_sw_sub_dofs_w;
    const double ib = lv.sup ? lv.sup_ib : 4.0;
    traced(h, "csr_resid_rows", m_all * (4 + 8 + 3 * wv) + (x_zero_first ? 0.0 : nnz_all * (ib + w)), [&] {
        C::resid_rows(rows, gather, lv, O::val(lv), x, r, v.rloc, x_zero_first, h->st);
    });
    for (int32_t c = 0; c < lv.n_colors; ++c) {
        const int64_t r0 = lv.color_row0[c], r1 = lv.color_row0[c + 1], rm = lv.color_rmid[c];
        const int64_t i0 = lv.color_item0[c], i1 = lv.color_item0[c + 1];
        const int64_t s0 = lv.color_smid[c], ns = lv.color_sub0[c + 1] - lv.color_smid[c];
        if (r1 == r0) continue;
        if (i1 > i0) {
            const double gb = lv.color_m2[c] * w + (double)(rm - r0) * (4 + 3 * wv);
            traced(h, "sub_symv", gb, [&] {
                C::symv(i1 - i0, lv.d_items + 3 * i0, lv.d_sw_sub_off, lv.d_sw_tp_off, O::inv(lv), v.rloc,
                        lv.d_scr_off, v.scr, lv.chl, h->st);
            });
            const double fb = lv.color_scr[c] * wv + (double)(rm - r0) * (8 + 2 * wv);
            traced(h, "sub_finalize", fb, [&] {
                C::finalize_colour(lv, c, v.scr, scatter, x, h->st);
            });
        }
        if (ns > 0) {
            const double sb = lv.color_pk[c] * w + (double)(r1 - rm) * (4 + 3 * wv);
            traced(h, "small_sub", sb, [&] { C::small(lv, s0, ns, O::pk(lv), v.rloc, x, scatter, h->st); });
        }
    }
}

// Mixed-precision multiplicative Schwarz sweep (FP32 vectors): the local residuals
// use the FP64 operator entries (sums in FP64, rounded once), the local solves
// the FP32 factors X = L^{-1} of A_Omega as X^T (X r) with FP64 sums, in one pass
// over the factor tiles -- a product of a matrix with its own transpose, so the
// rounded local solve stays symmetric positive semidefinite; an FP32 copy of the
// explicit inverse does not (on operators whose spectrum spans more than FP32
// resolves, it becomes indefinite).
void sweep_factor(lsdd_hierarchy* h, Level& lv, const float* r, float* x, bool forward, bool x_zero_first) {
    VecSet<float>& v = lv.v32[0];
    for (int32_t cc = 0; cc < lv.n_colors; ++cc) {
        int32_t c = forward ? cc : lv.n_colors - 1 - cc;
        const int64_t r0 = lv.color_row0[c], r1 = lv.color_row0[c + 1], rm = lv.color_rmid[c];
        const int64_t i0 = lv.color_item0[c], i1 = lv.color_item0[c + 1];
        const int64_t s0 = lv.color_smid[c], ns = lv.color_sub0[c + 1] - lv.color_smid[c];
        if (r1 == r0) continue;
        const bool xz = x_zero_first && cc == 0;
        const double rb = lv.color_m[c] * (4 + 8 + 3 * 4.0) + (xz ? 0.0 : lv.color_nnz[c] * ((lv.sup ? lv.sup_ib : 4.0) + 8.0));
        traced(h, "csr_resid_rows", rb, [&] {
            Cyc<float, 1>::resid_colour<double>(lv, c, lv.d_val, x, r, v.rloc, xz, h->st);
        });
        const int64_t j0 = lv.color_ritem0[c], j1 = lv.color_ritem0[c + 1];
        if (j1 > j0) {
            const double gb = lv.color_m2[c] * 4.0 + (double)(rm - r0) * (4 + 3 * 4.0);
            traced(h, "sub_fact", gb, [&] {
                launch_sub_fact(j1 - j0, lv.d_row_items + 2 * j0, lv.d_sw_sub_off, lv.d_sw_tp_off, lv.d_tfac32,
                                v.rloc, lv.d_scr_off, v.scr, lv.chl, lv.fact_stash ? lv.color_stash[c] : 0, h->st);
            });
            traced(h, "sub_finalize", lv.color_scr[c] * 4.0 + (double)(rm - r0) * 16.0, [&] {
                Cyc<float, 1>::finalize_colour(lv, c, v.scr, lv.d_sw_sub_dofs, x, h->st);
            });
        }
        if (ns > 0) {
            const double sb = lv.color_pk[c] * 4.0 + (double)(r1 - rm) * (4 + 3 * 4.0);
            traced(h, "small_sub", sb, [&] {
                launch_small_sub<float, 1>(s0, ns, lv.d_sw_sub_off, lv.d_sw_sub_dofs, lv.d_sw_pk_off, lv.d_pkfac32,
                                           v.rloc, x, lv.small_m, h->st, true);
            });
        }
    }
}

template <typename T, int NR>
void sweep(lsdd_hierarchy* h, Level& lv, const T* r, T* x, bool forward, bool x_zero_first) {
    using O = LvOps<T>;
    using C = Cyc<T, NR>;
    if (lv.smoother == 1) {
        sweep_ras<T, NR>(h, lv, r, x, !forward, x_zero_first);
        return;
    }
    VecSet<T>& v = O::v(lv, NR > 1);
    const double w = (double)sizeof(T), wv = w * NR;
    if constexpr (std::is_same<T, float>::value && NR == 1) {
        if (h->cycle_prec == 2) {
            sweep_factor(h, lv, r, x, forward, x_zero_first);
            return;
        }
    }
    for (int32_t cc = 0; cc < lv.n_colors; ++cc) {
        int32_t c = forward ? cc : lv.n_colors - 1 - cc;
        const int64_t r0 = lv.color_row0[c], r1 = lv.color_row0[c + 1], rm = lv.color_rmid[c];
        const int64_t i0 = lv.color_item0[c], i1 = lv.color_item0[c + 1];
        const int64_t s0 = lv.color_smid[c], ns = lv.color_sub0[c + 1] - lv.color_smid[c];
        if (r1 == r0) continue;
        const bool xz = x_zero_first && cc == 0;
        const double rb = lv.color_m[c] * (4 + 8 + 3 * wv) +
                          (xz ? 0.0 : lv.color_nnz[c] * ((lv.sup ? lv.sup_ib : 4.0) + w));
        traced(h, "csr_resid_rows", rb, [&] {
            C::template resid_colour<T>(lv, c, O::val(lv), x, r, v.rloc, xz, h->st);
        });
        if (i1 > i0) {
            const double gb = lv.color_m2[c] * w + (double)(rm - r0) * (4 + 3 * wv);
            traced(h, "sub_symv", gb, [&] {
                C::symv(i1 - i0, lv.d_items + 3 * i0, lv.d_sw_sub_off, lv.d_sw_tp_off, O::inv(lv), v.rloc,
                        lv.d_scr_off, v.scr, lv.chl, h->st);
            });
            const double fb = lv.color_scr[c] * wv + (double)(rm - r0) * (8 + 2 * wv);
            traced(h, "sub_finalize", fb, [&] {
                C::finalize_colour(lv, c, v.scr, lv.d_sw_sub_dofs, x, h->st);
            });
        }
        if (ns > 0) {
            const double sb = lv.color_pk[c] * w + (double)(r1 - rm) * (4 + 3 * wv);
            traced(h, "small_sub", sb, [&] { C::small(lv, s0, ns, O::pk(lv), v.rloc, x, lv.d_sw_sub_dofs, h->st); });
        }
    }
}

// Terminal blocks of a level in FP64: x[T] = A_T^{-1} r[T] for every block T
// (r, x level vectors of NR interleaved right-hand sides; x is written only on
// the blocks' DOFs).
template <int NR>
void terminal_solve(lsdd_hierarchy* h, Level& lv, const double* r, double* x) {
    using CD = Cyc<double, NR>;
    constexpr int b = NR > 1 ? 1 : 0;
    VecSet<double>& v = lv.v64[b];
    const double* rr = r;
    if (lv.c_dofs) {
        CD::resid_rows(lv.term_len, lv.c_dofs, lv, lv.d_val, r, r, v.rloc, true, h->st);   // gather
        rr = v.rloc;
    }
    const double nb = lv.c_entries * 8.0 + 2.0 * lv.term_len * 8.0 * NR;
    traced(h, "coarse_symv", nb, [&] {
        CD::symv(lv.c_nitems, lv.c_items, lv.c_sub_off, lv.c_tp_off, lv.c_tiles, rr, lv.c_scr_off, v.scr, lv.c_chl,
                 h->st);
    });
    CD::finalize(0, lv.term_len, lv.c_pos, lv.c_sub_off, lv.c_scr_off, v.scr, lv.c_dofs, x, false, lv.c_chl, 32,
                 h->st);
}

template <typename T, int NR>
void vcycle(lsdd_hierarchy* h, size_t l, const T* r, T* x) {
    using O = LvOps<T>;
    using C = Cyc<T, NR>;
    constexpr int b = NR > 1 ? 1 : 0;
    Level& lv = *h->L[l];
    const double w = (double)sizeof(T), wv = w * NR;
    // terminal blocks (all of the coarsest level) in FP64
    auto terminal = [&] {
        if constexpr (std::is_same<T, double>::value) {
            terminal_solve<NR>(h, lv, r, x);
        } else {
            launch_to_f64(lv.n * NR, r, lv.cr64[b], h->st);
            if (!lv.coarsest) launch_zero<double>(lv.n * NR, lv.cx64[b], h->st);
            terminal_solve<NR>(h, lv, lv.cr64[b], lv.cx64[b]);
            launch_to_f32(lv.n * NR, lv.cx64[b], x, h->st);
        }
    };
    if (lv.coarsest) {
        terminal();
        return;
    }
    Level& nx = *h->L[l + 1];
    VecSet<T>& v = O::v(lv, b);
    VecSet<T>& vn = O::v(nx, b);
    launch_zero<T>(lv.n * NR, x, h->st);
    if (!lv.term.empty()) terminal();     // instances whose hierarchy ends on this level
    sweep<T, NR>(h, lv, r, x, true, true);
    bool mixed = false;
    if constexpr (std::is_same<T, float>::value && NR == 1) {
        if (h->cycle_prec == 2) {
            mixed = true;
            traced(h, "csr_spmv", full_apply_bytes(lv, 8.0, wv, true), [&] {
                if (lv.eapply && lv.d_etri)
                    launch_elem_apply<float, double>(lv.el.count(), lv.d_elem_ptr, lv.d_elem_dofs, lv.d_etri_off,
                                                     lv.d_etri, lv.e_nmax, x, lv.d_ebuf, lv.n, lv.d_d2e_ptr, lv.d_e2y,
                                                     r, v.t, h->st);
                else
                    launch_csr_spmv<float, double>(lv.n, lv.d_rowptr, lv.sup ? lv.d_scol : lv.d_col, lv.d_val, x, v.t,
                                                   r, lv.lanes, h->st, lv.sup ? lv.d_scoff : nullptr);
            });
        }
    }
    if (!mixed)
        traced(h, "csr_spmv",
               NR == 1 ? full_apply_bytes(lv, w, wv, true)
                       : (double)lv.nnz * ((lv.sup ? lv.sup_ib : 4.0) + w) + (double)lv.n * (8 + 3 * wv),
               [&] { C::spmv(lv, O::val(lv), x, v.t, r, h->st); });
    const double zb = (double)lv.zoff.back() * w + (double)lv.n * (4 + wv) + (double)nx.n * wv;
    traced(h, "restrict", zb, [&] { C::restrict_(lv, O::Z(lv), v.t, vn.r, h->st); });
    vcycle<T, NR>(h, l + 1, vn.r, vn.x);
    traced(h, "prolong", zb + (double)lv.n * wv, [&] { C::prolong(lv, O::Z(lv), vn.x, x, h->st); });
    sweep<T, NR>(h, lv, r, x, false, false);
}

// block vectors of every level, on first use
void ensure_block_vectors(lsdd_hierarchy* h) {
    for (auto& lp : h->L)
        if (!lp->v64[1].r) alloc_vectors(h, *lp, 1);
}

template <int NR>
void precond(lsdd_hierarchy* h, const double* r, double* z) {
    Level& l0 = *h->L[0];
    constexpr int b = NR > 1 ? 1 : 0;
    if (h->cycle_prec >= 1) {
        launch_to_f32(l0.n * NR, r, l0.v32[b].r, h->st);
        vcycle<float, NR>(h, 0, l0.v32[b].r, l0.v32[b].x);
        launch_to_f64(l0.n * NR, l0.v32[b].x, z, h->st);
    } else {
        vcycle<double, NR>(h, 0, r, z);
    }
}

// ---------------------------------------------------------------- PCG

void alloc_pcg(lsdd_hierarchy* h, int b) {
    Arena& a = h->arena;
    const int64_t len = h->L[0]->n * (b ? NRB : 1);
    auto& B = h->pb[b];
    B.B = a.alloc<double>(len);
    B.X = a.alloc<double>(len);
    B.r = a.alloc<double>(len);
    B.p = a.alloc<double>(len);
    B.q = a.alloc<double>(len);
    B.z = a.alloc<double>(len);
    B.rold = a.alloc<double>(len);
}

// Segment table: DOF ranges [seg_off[s], seg_off[s+1]) cut into reduction
// blocks of at most 2048 DOFs.
void init_segments(lsdd_hierarchy* h, const std::vector<int64_t>& seg_off) {
    Arena& a = h->arena;
    const int32_t ns = (int32_t)seg_off.size() - 1;
    constexpr int64_t CH = 2048;
    std::vector<int32_t> bseg, sblk(1, 0);
    std::vector<int64_t> blo, bhi;
    for (int32_t s = 0; s < ns; ++s) {
        if (seg_off[s + 1] <= seg_off[s]) throw Error(LSDD_E_INVAL, "empty segment");
        for (int64_t d = seg_off[s]; d < seg_off[s + 1]; d += CH) {
            bseg.push_back(s);
            blo.push_back(d);
            bhi.push_back(std::min(d + CH, seg_off[s + 1]));
        }
        sblk.push_back((int32_t)bseg.size());
    }
    h->seg_off = seg_off;
    h->seg.n_seg = ns;
    h->seg.n_blk = (int32_t)bseg.size();
    h->seg.blk_seg = a.upload(bseg, h->st);
    h->seg.blk_lo = a.upload(blo, h->st);
    h->seg.blk_hi = a.upload(bhi, h->st);
    h->seg.seg_blk = a.upload(sblk, h->st);
    h->nsm = ns * NRB;
    h->sc = a.alloc<double>((size_t)9 * h->nsm);
    h->ic = a.alloc<int32_t>((size_t)2 * h->nsm + 4);
    h->part = a.alloc<double>((size_t)2 * h->seg.n_blk * NRB);
    if (!h->h_ic) HIPCHK(hipHostMalloc((void**)&h->h_ic, 4 * sizeof(int32_t), hipHostMallocDefault));
}

void reset_graphs(lsdd_hierarchy* h) {
    for (auto& a : h->gx)
        for (auto& b : a)
            for (auto& g : b)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
}

// PCG (x0 = 0) on the NR right-hand sides in pb[b].B, one recurrence per
// (segment, right-hand side) pair, preconditioned by one V-cycle; the solution
// is left in pb[b].X.  Returns true on breakdown.  Every scalar stays on the
// device; the host reads the active count once per iteration.
template <int NR>
bool pcg_run(lsdd_hierarchy* h) {
    constexpr int b = NR > 1 ? 1 : 0;
    auto& B = h->pb[b];
    hipStream_t st = h->st;
    Level& l0 = *h->L[0];
    const int64_t n = l0.n;
    const SegTable& T = h->seg;
    const int ns = T.n_seg * NR, nsm = h->nsm;
    double *bb = h->sc, *rz = bb + nsm, *pq = rz + nsm, *rr = pq + nsm, *rzn = rr + nsm, *rzo = rzn + nsm,
           *alpha = rzo + nsm, *beta = alpha + nsm, *relres = beta + nsm;
    int32_t *act = h->ic, *iters = act + nsm, *cnt = iters + nsm, *itf = cnt + 1;   // itf[0] it, itf[1] flag
    const bool flex = h->cycle_prec >= 1;
    const double tol2 = h->prm.rtol * h->prm.rtol;
    launch_seg_dot(T, NR, B.B, B.B, nullptr, nullptr, h->part, bb, nullptr, st);
    launch_pcg_init(ns, bb, act, iters, relres, itf, st);
    launch_pcg_start(n * NR, B.B, B.r, B.X, st);
    precond<NR>(h, B.r, B.z);
    launch_copy(n * NR, B.z, B.p, st);
    launch_seg_dot(T, NR, B.r, B.z, nullptr, nullptr, h->part, rz, nullptr, st);
    auto half_a = [&] {
        traced(h, "pcg_spmv",
               NR == 1 ? full_apply_bytes(l0, 8.0, 8.0, false)
                       : (double)l0.nnz * ((l0.sup ? l0.sup_ib : 4.0) + 8.0) + (double)n * 8.0 * (1 + 2 * NR),
               [&] { Cyc<double, NR>::spmv(l0, l0.d_val, B.p, B.q, nullptr, st); });
        launch_seg_dot(T, NR, B.p, B.q, nullptr, nullptr, h->part, pq, nullptr, st);
        launch_pcg_alpha(ns, act, rz, pq, alpha, itf + 1, st);
        if (flex) launch_copy(n * NR, B.r, B.rold, st);
        launch_pcg_update_xr(T, NR, act, alpha, B.p, B.q, B.X, B.r, h->part, rr, st);
        launch_pcg_check(ns, itf, tol2, bb, rr, act, iters, relres, cnt, itf + 1, st);
    };
    auto half_b = [&] {
        precond<NR>(h, B.r, B.z);
        launch_seg_dot(T, NR, B.r, B.z, flex ? B.rold : nullptr, flex ? B.z : nullptr, h->part, rzn, rzo, st);
        launch_pcg_beta(ns, act, rzn, flex ? rzo : nullptr, rz, beta, itf + 1, st);
        launch_pcg_update_p(T, NR, act, beta, B.z, B.p, st);
    };
    auto run = [&](int half, auto&& fn) {
        if (!h->use_graph || h->tr.on || !st) {
            fn();
            return;
        }
        hipGraphExec_t& g = h->gx[b][h->cycle_prec][half];
        if (!g) {
            hipGraph_t gr;
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            fn();
            HIPCHK(hipStreamEndCapture(st, &gr));
            HIPCHK(hipGraphInstantiate(&g, gr, nullptr, nullptr, 0));
            HIPCHK(hipGraphDestroy(gr));
        }
        HIPCHK(hipGraphLaunch(g, st));
    };
    bool breakdown = false;
    for (int it = 1; it <= h->prm.max_iter; ++it) {
        run(0, half_a);
        HIPCHK(hipMemcpyAsync(h->h_ic, cnt, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        sync(st);
        if (h->tr.on) h->tr.flush();
        if (h->h_ic[2]) {
            breakdown = true;
            h->breakdown_bits = h->h_ic[2];
            break;
        }
        if (h->h_ic[0] == 0) break;
        run(1, half_b);
    }
    HIPCHK(hipGetLastError());
    return breakdown;
}

// ---------------------------------------------------------------- autotuner

// Rebuild the work items and the partial-sum layout of the tiled subdomain
// product of a level for `chl` tiles per item.
void set_chunk(lsdd_hierarchy* h, Level& lv, int chl) {
    Arena& ar = h->arena;
    const int32_t n_sub = (int32_t)lv.sw_sub_off.size() - 1;
    lv.chl = chl;
    std::vector<int32_t> items;
    lv.color_item0.assign(lv.n_colors + 1, 0);
    for (int32_t c = 0; c < lv.n_colors; ++c) {
        std::vector<int32_t> subs;
        for (int32_t q = lv.color_sub0[c]; q < lv.color_smid[c]; ++q) subs.push_back(q);
        append_symv_items(lv.sw_sub_off, subs, chl, items);
        lv.color_item0[c + 1] = (int64_t)items.size() / 3;
    }
    std::vector<int64_t> scr_off(n_sub + 1, 0);
    lv.color_scr.assign(lv.n_colors, 0.0);
    for (int32_t q = 0; q < n_sub; ++q) {
        const int64_t m = lv.sw_sub_off[q + 1] - lv.sw_sub_off[q];
        scr_off[q + 1] = scr_off[q] + (m <= SMALL_M ? 0 : sub_symv_scratch_len(m, chl));
        lv.color_scr[lv.colors[lv.sweep[q]]] += (double)(scr_off[q + 1] - scr_off[q]);
    }
    ar.release(lv.d_items);
    ar.release(lv.d_scr_off);
    lv.d_items = ar.upload(items, h->st);
    lv.d_scr_off = ar.upload(scr_off, h->st);
    const int64_t need = std::max<int64_t>({scr_off[n_sub], lv.c_scr_len, 1});
    if (need > std::max<int64_t>({lv.scr_len, lv.c_scr_len, 1})) {
        for (int b = 0; b < 2; ++b) {
            const int64_t w = b ? NRB : 1;
            if (lv.v64[b].scr) {
                ar.release(lv.v64[b].scr);
                lv.v64[b].scr = ar.alloc<double>(need * w);
            }
            if (lv.v32[b].scr) {
                ar.release(lv.v32[b].scr);
                lv.v32[b].scr = ar.alloc<float>(need * w);
            }
        }
    }
    lv.scr_len = scr_off[n_sub];
    build_fin_tab(h, lv, scr_off);
    sync(h->st);
}

template <class F>
double time_ms(lsdd_hierarchy* h, F&& fn, int reps = 5) {
    // fastest of `reps` separately timed runs after a warm-up: the minimum is the
    // least noisy estimate of a candidate's own cost
    fn();
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    float best = 3.0e38f;
    for (int r = 0; r < reps; ++r) {
        HIPCHK(hipEventRecord(a, h->st));
        fn();
        HIPCHK(hipEventRecord(b, h->st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

// Time the candidates of every per-level launch shape on the level's own data
// and keep the fastest.  Values in the work vectors are irrelevant (zeroed).
template <typename T, int NR>
void autotune_levels(lsdd_hierarchy* h) {
    using O = LvOps<T>;
    using C = Cyc<T, NR>;
    constexpr int b = NR > 1 ? 1 : 0;
    for (auto& lp : h->L) {
        Level& lv = *lp;
        if (lv.coarsest) continue;
        VecSet<T>& v = O::v(lv, b);
        launch_zero<T>(lv.n * NR, v.r, h->st);
        launch_zero<T>(lv.n * NR, v.x, h->st);
        int& lanes = NR > 1 ? lv.lanes_b : lv.lanes;
        const std::vector<int> lane_c = NR > 1 ? std::vector<int>{4, 8, 16, 32, 64} : std::vector<int>{8, 16, 32, 64};
        double best = 1e300;
        int pick = lanes, pick_sup = 0;
        double best_row = 1e300;   // the per-row kernels' best lane count: it also serves the
        int pick_row = lanes;      // full products and the RAS sweep when row blocks win
        const int prev_sup = lv.sup;
        // a supernode-blocked level: also with the shared column lists and, for single
        // vectors, by supernode row blocks of 1, 2 or 4 waves
        std::vector<int> sup_c{0};
        if (lv.d_scoff) sup_c.push_back(1);
        if (lv.d_scoff && lv.d_rblk) {
            if (NR == 1) sup_c.insert(sup_c.end(), {2, 3, 4});
            else sup_c.push_back(2);   // blocks of right-hand sides: 4, 8 or 16 lanes per row block
        }
        for (int sp : sup_c) {
            lv.sup = sp;
            for (int L : lane_c) {
                lanes = L;
                const double ms = time_ms(h, [&] {
                    for (int32_t c = 0; c < lv.n_colors; ++c)
                        C::template resid_colour<T>(lv, c, O::val(lv), v.x, v.r, v.rloc, false, h->st);
                });
                if (sp >= 2 && NR > 1) {
                    vlog("autotune level %d: supernode row blocks, %d lanes each: %.3f ms", lv.level, L, ms);
                    if (ms < best) best = ms, pick = L, pick_sup = sp;
                    if (L >= 16) break;
                    continue;
                }
                if (sp >= 2) {
                    vlog("autotune level %d: supernode row blocks, %d wave(s) each: %.3f ms", lv.level,
                         1 << (sp - 2), ms);
                    if (ms < best) best = ms, pick_sup = sp;
                    break;
                }
                vlog("autotune level %d: CSR lanes %d%s: %.3f ms", lv.level, L, sp ? ", shared column lists" : "", ms);
                if (ms < best) best = ms, pick = L, pick_sup = sp;
                if (ms < best_row) best_row = ms, pick_row = L;
            }
        }
        lanes = (NR == 1 && pick_sup >= 2) ? pick_row : pick;
        // one setting serves both: blocks of right-hand sides that choose row blocks keep
        // the single vectors' choice of waves per block
        lv.sup = (NR > 1 && pick_sup >= 2 && prev_sup >= 2) ? prev_sup : pick_sup;
        if (NR == 1 && build_elem_apply(h, lv)) {
            // the full product (pre-restriction residual, PCG) from the CSR or the element triangles
            best = 1e300;
            int pick_e = 0;
            for (int ea : {0, 1}) {
                lv.eapply = ea;
                const double ms = time_ms(h, [&] { C::spmv(lv, O::val(lv), v.x, v.t, v.r, h->st); });
                vlog("autotune level %d: full product from %s: %.3f ms", lv.level, ea ? "element triangles" : "CSR", ms);
                if (ms < best) best = ms, pick_e = ea;
            }
            lv.eapply = pick_e;
        }
        if (lv.color_item0.back() == 0) continue;   // no large overlap on this level
        auto run_large = [&] {
            for (int32_t c = 0; c < lv.n_colors; ++c) {
                const int64_t i0 = lv.color_item0[c], i1 = lv.color_item0[c + 1];
                if (i1 == i0) continue;
                C::symv(i1 - i0, lv.d_items + 3 * i0, lv.d_sw_sub_off, lv.d_sw_tp_off, O::inv(lv), v.rloc,
                        lv.d_scr_off, v.scr, lv.chl, h->st);
                C::finalize_colour(lv, c, v.scr, lv.d_sw_sub_dofs, v.x, h->st);
            }
        };
        best = 1e300;
        int pick_chl = lv.chl;
        for (int chl : {2, 4, 8}) {
            set_chunk(h, lv, chl);
            const double ms = time_ms(h, run_large);
            vlog("autotune level %d: %d tiles per item: %.3f ms", lv.level, chl, ms);
            if (ms < best) best = ms, pick_chl = chl;
        }
        set_chunk(h, lv, pick_chl);
        best = 1e300;
        int pick_fl = lv.fl;
        for (int fl : {8, 32}) {
            lv.fl = fl;
            const double ms = time_ms(h, run_large);
            vlog("autotune level %d: finalize threads per DOF %d: %.3f ms", lv.level, fl, ms);
            if (ms < best) best = ms, pick_fl = fl;
        }
        lv.fl = pick_fl;
        if constexpr (std::is_same<T, float>::value && NR == 1) {
            if (h->cycle_prec == 2 && lv.d_row_items) {
                // the mixed cycle's factor product, with and without the tile rows kept in LDS
                auto run_fact = [&] {
                    for (int32_t c = 0; c < lv.n_colors; ++c) {
                        const int64_t j0 = lv.color_ritem0[c], j1 = lv.color_ritem0[c + 1];
                        if (j1 == j0) continue;
                        launch_sub_fact(j1 - j0, lv.d_row_items + 2 * j0, lv.d_sw_sub_off, lv.d_sw_tp_off,
                                        lv.d_tfac32, v.rloc, lv.d_scr_off, v.scr, lv.chl,
                                        lv.fact_stash ? lv.color_stash[c] : 0, h->st);
                        C::finalize_colour(lv, c, v.scr, lv.d_sw_sub_dofs, v.x, h->st);
                    }
                };
                best = 1e300;
                int pick_fs = lv.fact_stash;
                for (int fs : {0, 1}) {
                    lv.fact_stash = fs;
                    const double ms = time_ms(h, run_fact);
                    vlog("autotune level %d: factor product, rows %s: %.3f ms", lv.level, fs ? "kept in LDS" : "re-read", ms);
                    if (ms < best) best = ms, pick_fs = fs;
                }
                lv.fact_stash = pick_fs;
            }
        }
    }
    sync(h->st);
}

// ---------------------------------------------------------------- setup driver

// Rows of a black-box CSR Gram factor as level-0 elements: element e is the row whose
// values start at val + src_off[e] (val on the host or the device).
struct GramCsrRows {
    std::vector<int64_t> src_off;
    const double* val = nullptr;
    bool on_device = false;
    int64_t nnz = 0;
};

lsdd_hierarchy* build(ElemList el0, const double* blocks, bool blocks_on_device, const GramCsrRows* gram_rows,
                      int64_t n, const int32_t* node_of_dof, const int32_t* agg_of_dof, const lsdd_params* prm,
                      void* stream, std::vector<int64_t> inst_off = {}, const double* elem_scale = nullptr) {
    auto h = std::make_unique<lsdd_hierarchy>();
    lsdd_params_default(&h->prm);
    if (prm) h->prm = *prm;
    const lsdd_params& P = h->prm;
    if (P.max_levels < 1 || P.precision < 0 || P.precision > 2 || P.tau_const <= 0 || P.rtol <= 0 || P.max_iter < 1 ||
        P.closure < 0 || P.closure > 1 || !(P.closure_tol >= 0) || P.smoother < 0 || P.smoother > 2 ||
        P.elem_factor < 0 || P.elem_factor > 1 || P.galerkin_precision < 0 || P.galerkin_precision > 1)
        throw Error(LSDD_E_INVAL, "invalid parameters");
    h->st = (hipStream_t)stream;
    double t0 = now_s();
    auto lv = std::make_unique<Level>();
    lv->level = 0;
    lv->n = n;
    lv->el = std::move(el0);
    lv->inst_off = inst_off.empty() ? std::vector<int64_t>{0, n} : inst_off;
    const int64_t ne = lv->el.count();
    lv->blk_off.assign(ne + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        int64_t s = lv->el.ptr[e + 1] - lv->el.ptr[e];
        lv->blk_off[e + 1] = lv->blk_off[e] + s * s;
    }
    if (node_of_dof) {
        lv->node_of_dof.assign(node_of_dof, node_of_dof + n);
        int32_t mx = -1;
        for (int32_t v : lv->node_of_dof) {
            if (v < 0) throw Error(LSDD_E_INVAL, "negative supernode id");
            mx = std::max(mx, v);
        }
        std::vector<char> used(mx + 1, 0);
        for (int32_t v : lv->node_of_dof) used[v] = 1;
        for (char u : used)
            if (!u) throw Error(LSDD_E_INVAL, "supernode ids must be 0..n_super-1, each used");
        lv->n_super = mx + 1;
    } else {
        lv->node_of_dof.resize(n);
        for (int64_t d = 0; d < n; ++d) lv->node_of_dof[d] = (int32_t)d;
        lv->n_super = (int32_t)n;
    }
    Arena& ar = h->arena;
    upload_elements(h.get(), *lv);
    lv->d_blocks = ar.alloc<double>(lv->blk_off[ne]);
    if (!gram_rows)
        HIPCHK(hipMemcpyAsync(lv->d_blocks, blocks, lv->blk_off[ne] * sizeof(double),
                              blocks_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->st));
    if (elem_scale) {
        // A_e = theta_e A_e^(1): scale the blocks on the device, keep theta for lsdd_update_theta
        h->d_scale0 = ar.alloc<double>(ne);
        HIPCHK(hipMemcpyAsync(h->d_scale0, elem_scale, ne * sizeof(double),
                              blocks_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->st));
        launch_scale_blocks(ne, lv->d_blk_off, h->d_scale0, lv->d_blocks, h->st);
    }
    // element Gram factors (Sec. 5.2)
    lv->d_G = ar.alloc<double>(lv->blk_off[ne]);
    if (!gram_rows) {
        int32_t* d_ranks = ar.alloc<int32_t>(ne);
        int32_t* d_status = ar.alloc<int32_t>(ne);
        int64_t max_ne = 0;
        for (int64_t e = 0; e < ne; ++e) max_ne = std::max(max_ne, lv->el.ptr[e + 1] - lv->el.ptr[e]);
        const int64_t stride = std::max<int64_t>(3 * max_ne * max_ne, elem_eig_scratch_stride(max_ne));
        // process elements in chunks so the eigen scratch stays bounded
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(ne, (int64_t(1) << 30) / (stride * 8)));
        double* scratch = ar.alloc<double>(chunk * stride);
        for (int64_t e0 = 0; e0 < ne; e0 += chunk) {
            int64_t cnt = std::min(chunk, ne - e0);
            if (P.elem_factor == 1)
                launch_elem_pchol(cnt, lv->d_elem_ptr + e0, lv->d_blk_off + e0, lv->d_blocks, lv->d_G,
                                  d_ranks + e0, d_status + e0, scratch, stride, P.rank_rtol, P.spsd_tol, h->st);
            else
                launch_elem_eig(cnt, lv->d_elem_ptr + e0, lv->d_blk_off + e0, lv->d_blocks, lv->d_G, d_ranks + e0,
                                d_status + e0, scratch, stride, P.rank_rtol, P.spsd_tol, max_ne, h->st);
        }
        HIPCHK(hipGetLastError());
        std::vector<int32_t> status = download(d_status, ne, h->st);
        lv->ranks = download(d_ranks, ne, h->st);
        vlog("element Gram factors for %lld elements %.3f s", (long long)ne, now_s() - t0);
        for (int64_t e = 0; e < ne; ++e) {
            if (status[e] == 1) throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + ": block is not symmetric or not finite");
            if (status[e] == 2) throw Error(LSDD_E_NOT_SPSD, "element " + std::to_string(e) + ": block is not SPSD");
        }
        ar.release(scratch);
        ar.release(d_ranks);
        ar.release(d_status);
    } else {
        // CSR G input: the Gram row is the element factor and the block is g^T g, both
        // formed on the device from the row values
        lv->ranks.assign(ne, 1);
        int64_t* d_src = ar.upload(gram_rows->src_off, h->st);
        const double* d_val = gram_rows->val;
        double* d_copy = nullptr;
        if (!gram_rows->on_device) {
            d_copy = ar.alloc<double>(std::max<int64_t>(gram_rows->nnz, 1));
            HIPCHK(hipMemcpyAsync(d_copy, gram_rows->val, gram_rows->nnz * sizeof(double), hipMemcpyHostToDevice,
                                  h->st));
            d_val = d_copy;
        }
        int32_t* d_fin = ar.alloc<int32_t>(1);
        HIPCHK(hipMemsetAsync(d_fin, 0, sizeof(int32_t), h->st));
        launch_check_finite(gram_rows->nnz, d_val, d_fin, h->st);
        if (download(d_fin, 1, h->st)[0]) throw Error(LSDD_E_INVAL, "non-finite value in G");
        launch_gram_csr_rows(ne, lv->d_elem_ptr, d_src, lv->d_blk_off, d_val, lv->d_G, lv->d_blocks, h->st);
        HIPCHK(hipGetLastError());
        sync(h->st);
        for (void* q : {(void*)d_src, (void*)d_copy, (void*)d_fin})
            if (q) ar.release(q);
    }
    const double tas = now_s();
    assemble_operator(h.get(), *lv);
    HIPCHK(hipGetLastError());
    sync(h->st);
    vlog("level 0: operator assembly %.3f s (setup so far %.3f s)", now_s() - tas, now_s() - t0);
    h->L.push_back(std::move(lv));
    while (true) {
        Level& cur = *h->L.back();
        // stopping tests per instance (one instance: the level itself); an
        // instance that stops here gets its terminal block on this level
        const int32_t n_inst = (int32_t)cur.inst_off.size() - 1;
        std::vector<int32_t> term, active;
        for (int32_t i = 0; i < n_inst; ++i) {
            const int64_t a = cur.inst_off[i], b = cur.inst_off[i + 1];
            if (b == a) continue;                       // ended on a finer level
            const double ni = (double)(b - a);
            const double density = (double)(cur.pat.ptr[b] - cur.pat.ptr[a]) / (ni * ni);
            const bool last = (int)h->L.size() >= P.max_levels || ni < P.min_coarse || density > P.max_density;
            (last ? term : active).push_back(i);
        }
        if (active.empty()) {
            make_terminal(h.get(), cur, term, true);
            break;
        }
        if (!term.empty()) make_terminal(h.get(), cur, term, false);
        std::unique_ptr<Level> nxt = coarsen(h.get(), cur, cur.level == 0 ? agg_of_dof : nullptr);
        if (!nxt) {
            // no mode retained anywhere: every instance present ends here
            std::vector<int32_t> all(term);
            all.insert(all.end(), active.begin(), active.end());
            std::sort(all.begin(), all.end());
            make_terminal(h.get(), cur, all, true);
            break;
        }
        h->L.push_back(std::move(nxt));
    }
    init_segments(h.get(), h->L[0]->inst_off);
    alloc_pcg(h.get(), 0);
    sync(h->st);
    h->setup_s = now_s() - t0;
    vlog("setup %.3f s", h->setup_s);
    h->cycle_prec = P.precision;
    return h.release();
}

}  // namespace
}  // namespace lsdd

using namespace lsdd;

// ====================================================================== C-ABI

extern "C" {

void lsdd_params_default(lsdd_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->max_levels = 3;
    p->agg_passes = 2;
    p->agg_passes_coarse = 1;
    p->modes_fixed = 0;
    p->min_coarse = 10;
    p->max_iter = 1000;
    p->precision = 0;
    p->tau_const = 0.75;
    p->max_density = 0.25;
    p->rtol = 1e-8;
    p->cluster_tol = 1e-9;
    p->band_tol = 1e-9;
    p->rank_rtol = 0.0;
    p->spsd_tol = 1e-12;
    p->closure = 0;
    p->closure_tol = 1e-12;
}

const char* lsdd_last_error(void) { return g_err.c_str(); }

void lsdd_set_allocator(lsdd_alloc_fn alloc, lsdd_free_fn free_fn, void* ctx) {
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_ctx = ctx;
}

#define ABI_BEGIN \
    g_err.clear(); \
    try {
#define ABI_END                                  \
    }                                            \
    catch (const Error& e) {                     \
        g_err = e.what();                        \
        return e.code;                           \
    }                                            \
    catch (const std::bad_alloc&) {              \
        g_err = "host allocation failed";        \
        return LSDD_E_NOMEM;                     \
    }                                            \
    catch (const std::exception& e) {            \
        g_err = e.what();                        \
        return LSDD_E_INVAL;                     \
    }

lsdd_status lsdd_setup_elements_scaled(int64_t n, int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                                       const double* elem_blocks, const double* elem_scale,
                                       const int32_t* node_of_dof, const int32_t* agg_of_dof, int mem_is_device,
                                       const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out);

lsdd_status lsdd_setup_elements(int64_t n, int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                                const double* elem_blocks, const int32_t* node_of_dof, const int32_t* agg_of_dof,
                                int mem_is_device, const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out) {
    return lsdd_setup_elements_scaled(n, n_elem, elem_ptr, elem_dofs, elem_blocks, nullptr, node_of_dof, agg_of_dof,
                                      mem_is_device, params, hip_stream, out);
}

lsdd_status lsdd_setup_elements_scaled(int64_t n, int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                                       const double* elem_blocks, const double* elem_scale,
                                       const int32_t* node_of_dof, const int32_t* agg_of_dof, int mem_is_device,
                                       const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out) {
    ABI_BEGIN
    if (!out) throw Error(LSDD_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t(1) << 31) || n_elem < 1 || !elem_ptr || !elem_dofs || !elem_blocks)
        throw Error(LSDD_E_INVAL, "bad sizes or NULL arrays");
    ElemList el;
    el.ptr.assign(elem_ptr, elem_ptr + n_elem + 1);
    if (el.ptr[0] != 0) throw Error(LSDD_E_INVAL, "elem_ptr[0] must be 0");
    std::vector<char> covered(n, 0), seen(n, 0);
    for (int64_t e = 0; e < n_elem; ++e) {
        int64_t s = el.ptr[e + 1] - el.ptr[e];
        if (s < 1 || s > 128) throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + " has " + std::to_string(s) + " DOFs (1..128 supported)");
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) {
            int32_t d = elem_dofs[q];
            if (d < 0 || d >= n) throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + ": DOF index out of range");
            if (seen[d]) throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + ": repeated DOF");
            seen[d] = 1;
            covered[d] = 1;
        }
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) seen[elem_dofs[q]] = 0;
    }
    for (int64_t d = 0; d < n; ++d)
        if (!covered[d]) throw Error(LSDD_E_INVAL, "DOF " + std::to_string(d) + " belongs to no element");
    el.dofs.assign(elem_dofs, elem_dofs + el.ptr[n_elem]);
    if (agg_of_dof) {
        int32_t mx = -1;
        for (int64_t d = 0; d < n; ++d) {
            if (agg_of_dof[d] < 0) throw Error(LSDD_E_INVAL, "negative aggregate id");
            mx = std::max(mx, agg_of_dof[d]);
        }
        std::vector<char> used(mx + 1, 0);
        for (int64_t d = 0; d < n; ++d) used[agg_of_dof[d]] = 1;
        for (char u : used)
            if (!u) throw Error(LSDD_E_INVAL, "aggregate ids must be 0..n_agg-1, each used");
    }
    *out = build(std::move(el), elem_blocks, mem_is_device != 0, nullptr, n, node_of_dof, agg_of_dof, params, hip_stream,
                 {}, elem_scale);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_update_theta(lsdd_hierarchy* h, const double* theta, void* hip_stream) {
    ABI_BEGIN
    if (!h || !theta) throw Error(LSDD_E_INVAL, "NULL argument");
    if (!h->L[0]->d_d2e_ptr) throw Error(LSDD_E_UNSUPPORTED, "the hierarchy was not built from element blocks");
    h->st = (hipStream_t)hip_stream;
    Level& l0 = *h->L[0];
    const int64_t ne = l0.el.count();
    if (!h->d_factor) h->d_factor = h->arena.alloc<double>(ne);
    launch_theta_factor(ne, theta, h->d_scale0, h->d_factor, h->st);
    HIPCHK(hipMemsetAsync(l0.d_val, 0, l0.nnz * sizeof(double), h->st));
    launch_assemble_rows(l0.n, l0.d_d2e_ptr, l0.d_d2e_elem, l0.d_d2e_loc, l0.d_elem_ptr, l0.d_elem_dofs, l0.d_blk_off,
                         l0.d_blocks, h->d_factor, l0.d_rowptr, l0.d_col, l0.d_val, h->st);
    if (l0.d_val32) launch_to_f32(l0.nnz, l0.d_val, l0.d_val32, h->st);
    if (l0.d_etri) pack_elem_tri(h, l0);
    HIPCHK(hipGetLastError());
    sync(h->st);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_elem_bilinear(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs, const double* blocks,
                               const double* u, const double* v, int32_t nrhs, int64_t ld, double scale, double* out,
                               void* hip_stream) {
    ABI_BEGIN
    if (n_elem < 1 || !elem_ptr || !elem_dofs || !blocks || !u || !v || !out || nrhs < 1 || ld < 1)
        throw Error(LSDD_E_INVAL, "bad argument");
    if (elem_ptr[0] != 0) throw Error(LSDD_E_INVAL, "elem_ptr[0] must be 0");
    std::vector<int64_t> boff(n_elem + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e) {
        const int64_t s = elem_ptr[e + 1] - elem_ptr[e];
        if (s < 1 || s > 4096) throw Error(LSDD_E_INVAL, "bad element size");
        boff[e + 1] = boff[e] + s * s;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    struct Scoped {
        Arena a;
        ~Scoped() { a.clear(); }
    } sc;
    const std::vector<int64_t> ptr(elem_ptr, elem_ptr + n_elem + 1);
    int64_t* d_ptr = sc.a.upload(ptr, st);
    int64_t* d_boff = sc.a.upload(boff, st);
    launch_elem_bilinear(n_elem, d_ptr, elem_dofs, d_boff, blocks, u, v, nrhs, ld, scale, out, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_setup_batched(int32_t n_inst, const int64_t* inst_n, const int64_t* inst_n_elem,
                               const int64_t* elem_ptr, const int32_t* elem_dofs, const double* elem_blocks,
                               const int32_t* node_of_dof, const int32_t* agg_of_dof, int mem_is_device,
                               const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out) {
    ABI_BEGIN
    if (!out) throw Error(LSDD_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_inst < 1 || !inst_n || !inst_n_elem || !elem_ptr || !elem_dofs || !elem_blocks)
        throw Error(LSDD_E_INVAL, "bad sizes or NULL arrays");
    std::vector<int64_t> inst_off(n_inst + 1, 0), elem_off(n_inst + 1, 0);
    for (int32_t i = 0; i < n_inst; ++i) {
        if (inst_n[i] < 1 || inst_n_elem[i] < 1) throw Error(LSDD_E_INVAL, "instance " + std::to_string(i) + " is empty");
        inst_off[i + 1] = inst_off[i] + inst_n[i];
        elem_off[i + 1] = elem_off[i] + inst_n_elem[i];
    }
    const int64_t n = inst_off[n_inst], n_elem = elem_off[n_inst];
    if (n >= (int64_t(1) << 31)) throw Error(LSDD_E_INVAL, "too many DOFs in the batch");
    if (elem_ptr[0] != 0) throw Error(LSDD_E_INVAL, "elem_ptr[0] must be 0");
    // union numbering: instance-local DOF, supernode and aggregate ids shifted by the instance offsets
    ElemList el;
    el.ptr.assign(elem_ptr, elem_ptr + n_elem + 1);
    el.dofs.resize(el.ptr[n_elem]);
    std::vector<char> covered(n, 0), seen(n, 0);
    for (int32_t i = 0; i < n_inst; ++i)
        for (int64_t e = elem_off[i]; e < elem_off[i + 1]; ++e) {
            const int64_t sz = el.ptr[e + 1] - el.ptr[e];
            if (sz < 1 || sz > 128)
                throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + " has " + std::to_string(sz) + " DOFs (1..128 supported)");
            for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) {
                const int32_t dl = elem_dofs[q];
                if (dl < 0 || dl >= inst_n[i])
                    throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + ": DOF index out of its instance's range");
                const int64_t d = inst_off[i] + dl;
                if (seen[d]) throw Error(LSDD_E_INVAL, "element " + std::to_string(e) + ": repeated DOF");
                seen[d] = 1;
                covered[d] = 1;
                el.dofs[q] = (int32_t)d;
            }
            for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) seen[el.dofs[q]] = 0;
        }
    for (int64_t d = 0; d < n; ++d)
        if (!covered[d]) throw Error(LSDD_E_INVAL, "DOF " + std::to_string(d) + " belongs to no element");
    auto shift = [&](const int32_t* v, const char* what) {
        std::vector<int32_t> u(n);
        int32_t base = 0;
        for (int32_t i = 0; i < n_inst; ++i) {
            int32_t mx = -1;
            for (int64_t d = inst_off[i]; d < inst_off[i + 1]; ++d) {
                if (v[d] < 0) throw Error(LSDD_E_INVAL, std::string("negative ") + what + " id");
                mx = std::max(mx, v[d]);
                u[d] = base + v[d];
            }
            std::vector<char> used(mx + 1, 0);
            for (int64_t d = inst_off[i]; d < inst_off[i + 1]; ++d) used[v[d]] = 1;
            for (char c : used)
                if (!c) throw Error(LSDD_E_INVAL, std::string(what) + " ids of an instance must be 0..count-1, each used");
            base += mx + 1;
        }
        return u;
    };
    std::vector<int32_t> nodes, aggs;
    if (node_of_dof) nodes = shift(node_of_dof, "supernode");
    if (agg_of_dof) aggs = shift(agg_of_dof, "aggregate");
    *out = build(std::move(el), elem_blocks, mem_is_device != 0, nullptr, n, node_of_dof ? nodes.data() : nullptr,
                 agg_of_dof ? aggs.data() : nullptr, params, hip_stream, inst_off);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_setup_gram_csr(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                                const int32_t* node_of_dof, const int32_t* agg_of_dof, int mem_is_device,
                                const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out) {
    ABI_BEGIN
    if (!out) throw Error(LSDD_E_INVAL, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || n >= (int64_t(1) << 31) || !rowptr || !col || !val) throw Error(LSDD_E_INVAL, "bad arguments");
    // the integer structure is read on the host (copied back once for device input)
    std::vector<int64_t> rp_h;
    std::vector<int32_t> col_h;
    const int64_t* rp = rowptr;
    const int32_t* cl = col;
    if (mem_is_device) {
        rp_h.resize(m + 1);
        HIPCHK(hipMemcpy(rp_h.data(), rowptr, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (rp_h[0] != 0 || rp_h[m] < 0) throw Error(LSDD_E_INVAL, "rowptr must start at 0 and end at nnz >= 0");
        col_h.resize(rp_h[m]);
        if (rp_h[m] > 0)
            HIPCHK(hipMemcpy(col_h.data(), col, rp_h[m] * sizeof(int32_t), hipMemcpyDeviceToHost));
        rp = rp_h.data();
        cl = col_h.data();
    }
    if (rp[0] != 0) throw Error(LSDD_E_INVAL, "rowptr must start at 0");
    ElemList el;
    el.ptr.assign(1, 0);
    GramCsrRows gr;
    std::vector<char> covered(n, 0);
    for (int64_t j = 0; j < m; ++j) {
        int64_t a = rp[j], b = rp[j + 1];
        if (b < a) throw Error(LSDD_E_INVAL, "rowptr not monotone");
        if (b == a) continue;                               // zero rows are dropped
        if (b - a > 128) throw Error(LSDD_E_UNSUPPORTED, "a row of G has more than 128 entries");
        for (int64_t q = a; q < b; ++q) {
            if (cl[q] < 0 || cl[q] >= n) throw Error(LSDD_E_INVAL, "column index out of range");
            covered[cl[q]] = 1;
            el.dofs.push_back(cl[q]);
        }
        gr.src_off.push_back(a);
        el.ptr.push_back((int64_t)el.dofs.size());
    }
    for (int64_t d = 0; d < n; ++d)
        if (!covered[d]) throw Error(LSDD_E_INVAL, "column " + std::to_string(d) + " of G is empty (A singular)");
    gr.val = val;
    gr.on_device = mem_is_device != 0;
    gr.nnz = rp[m];
    *out = build(std::move(el), nullptr, false, &gr, n, node_of_dof, agg_of_dof, params, hip_stream);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_destroy(lsdd_hierarchy* h) {
    ABI_BEGIN
    if (!h) return LSDD_OK;
    if (h->st) (void)hipStreamSynchronize(h->st);
    else (void)hipDeviceSynchronize();
    reset_graphs(h);
    h->tr.destroy();
    h->arena.clear();
    if (h->h_ic) (void)hipHostFree(h->h_ic);
    delete h;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_vcycle(lsdd_hierarchy* h, const double* r, double* z, void* hip_stream) {
    ABI_BEGIN
    if (!h || !r || !z) throw Error(LSDD_E_INVAL, "NULL argument");
    h->st = (hipStream_t)hip_stream;
    precond<1>(h, r, z);
    HIPCHK(hipGetLastError());
    sync(h->st);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_elem_bilinear_noalloc(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                                       const double* blocks, const double* u, const double* v, int32_t nrhs,
                                       int64_t ld, double scale, double* out, void* hip_stream) {
    ABI_BEGIN
    if (n_elem < 1 || !elem_ptr || !elem_dofs || !blocks || !u || !v || !out || nrhs < 1 || ld < 1)
        throw Error(LSDD_E_INVAL, "bad argument");
    if (n_elem > NOALLOC_MAX_ELEM)
        throw Error(LSDD_E_UNSUPPORTED, "lsdd_elem_bilinear_noalloc: more than 1048576 elements");
    if (elem_ptr[0] != 0) throw Error(LSDD_E_INVAL, "elem_ptr[0] must be 0");
    for (int64_t e = 0; e < n_elem; ++e) {
        const int64_t m = elem_ptr[e + 1] - elem_ptr[e];
        if (m < 1 || m > 4096) throw Error(LSDD_E_INVAL, "bad element size");
    }
    int64_t* scr = nullptr;
    HIPCHK(noalloc_scratch(&scr));
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t* d_ptr = scr;
    int64_t* d_boff = scr + (n_elem + 1);
    HIPCHK(hipMemcpyAsync(d_ptr, elem_ptr, (size_t)(n_elem + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    launch_block_offsets(n_elem, d_ptr, d_boff, st);
    launch_elem_bilinear(n_elem, d_ptr, elem_dofs, d_boff, blocks, u, v, nrhs, ld, scale, out, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return LSDD_OK;
    ABI_END
}
lsdd_status lsdd_apply(lsdd_hierarchy* h, int32_t level, const double* x, double* y, void* hip_stream) {
    ABI_BEGIN
    if (!h || !x || !y || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    h->st = (hipStream_t)hip_stream;
    Level& lv = *h->L[level];
    Cyc<double, 1>::spmv(lv, lv.d_val, x, y, nullptr, h->st);
    HIPCHK(hipGetLastError());
    sync(h->st);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_solve(lsdd_hierarchy* h, const double* b, double* x, int32_t nrhs, void* hip_stream, lsdd_info* info) {
    ABI_BEGIN
    if (!h || !b || !x || nrhs < 1) throw Error(LSDD_E_INVAL, "bad argument");
    if (nrhs > 1 && h->cycle_prec == 2) throw Error(LSDD_E_UNSUPPORTED, "the mixed cycle runs single right-hand sides only");
    h->st = (hipStream_t)hip_stream;
    hipStream_t st = h->st;
    const int64_t n = h->L[0]->n;
    const int32_t nseg = h->seg.n_seg;
    const double t0 = now_s();
    int32_t* fin = h->ic + 2 * h->nsm + 3;
    HIPCHK(hipMemsetAsync(fin, 0, sizeof(int32_t), st));
    launch_check_finite(n * nrhs, b, fin, st);
    if (download(fin, 1, st)[0]) throw Error(LSDD_E_INVAL, "right-hand side has NaN/Inf");
    std::vector<lsdd_info> out((size_t)nrhs * nseg);
    bool breakdown = false;
    auto collect = [&](int32_t k0, int32_t nr, int NR) {
        std::vector<int32_t> it = download(h->ic + h->nsm, (size_t)nseg * NR, st);
        std::vector<int32_t> act = download(h->ic, (size_t)nseg * NR, st);
        std::vector<double> rel = download(h->sc + 8 * (size_t)h->nsm, (size_t)nseg * NR, st);
        for (int32_t k = 0; k < nr; ++k)
            for (int32_t sg = 0; sg < nseg; ++sg) {
                const size_t i = (size_t)sg * NR + k;
                lsdd_info& f = out[(size_t)(k0 + k) * nseg + sg];
                f.iters = it[i];
                f.rel_res = rel[i];
                f.converged = (!act[i] && rel[i] <= h->prm.rtol) ? 1 : 0;
                f.setup_s = h->setup_s;
            }
    };
    if (nrhs == 1) {
        launch_copy(n, b, h->pb[0].B, st);
        breakdown = pcg_run<1>(h);
        launch_copy(n, h->pb[0].X, x, st);
        collect(0, 1, 1);
    } else {
        if (!h->pb[1].B) {
            ensure_block_vectors(h);
            alloc_pcg(h, 1);
        }
        for (int32_t k0 = 0; k0 < nrhs && !breakdown; k0 += NRB) {
            const int32_t nr = std::min<int32_t>(NRB, nrhs - k0);
            launch_gather_rhs(n, nr, b + (int64_t)k0 * n, n, h->pb[1].B, st);
            breakdown = pcg_run<NRB>(h);
            launch_scatter_sol(n, nr, h->pb[1].X, x + (int64_t)k0 * n, n, st);
            collect(k0, nr, NRB);
        }
    }
    HIPCHK(hipGetLastError());
    sync(st);
    const double ts = now_s() - t0;
    bool allconv = true;
    for (auto& f : out) {
        f.solve_s = ts;
        allconv = allconv && f.converged;
    }
    if (info) std::copy(out.begin(), out.end(), info);
    if (breakdown) throw Error(LSDD_E_BREAKDOWN, "PCG breakdown: " + breakdown_cause(h->breakdown_bits));
    if (!allconv) {
        g_err = "PCG did not reach rtol within max_iter";
        return LSDD_E_NOCONV;
    }
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_solve_batched(int32_t n_inst, lsdd_hierarchy* const* hs, const double* const* b, double* const* x,
                               int32_t nrhs, void* hip_stream, lsdd_info* info) {
    if (n_inst < 1 || !hs || !b || !x || nrhs < 1) {
        g_err = "bad argument";
        return LSDD_E_INVAL;
    }
    for (int32_t i = 0; i < n_inst; ++i)
        if (!hs[i] || !b[i] || !x[i]) {
            g_err = "NULL hierarchy or vector of instance " + std::to_string(i);
            return LSDD_E_INVAL;
        }
    int64_t off = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        const lsdd_status s = lsdd_solve(hs[i], b[i], x[i], nrhs, hip_stream, info ? info + off : nullptr);
        if (s != LSDD_OK) return s;
        off += (int64_t)nrhs * hs[i]->seg.n_seg;
    }
    return LSDD_OK;
}
lsdd_status lsdd_solve_stationary(lsdd_hierarchy* h, const double* b, double* x, int32_t nrhs, void* hip_stream,
                                  lsdd_info* info) {
    ABI_BEGIN
    if (!h || !b || !x || nrhs < 1) throw Error(LSDD_E_INVAL, "bad argument");
    if (h->seg.n_seg != 1)
        throw Error(LSDD_E_UNSUPPORTED, "the standalone cycle iteration needs a single-problem hierarchy");
    h->st = (hipStream_t)hip_stream;
    hipStream_t st = h->st;
    Level& l0 = *h->L[0];
    const int64_t n = l0.n;
    const double t0 = now_s();
    int32_t* fin = h->ic + 2 * h->nsm + 3;
    HIPCHK(hipMemsetAsync(fin, 0, sizeof(int32_t), st));
    launch_check_finite(n * nrhs, b, fin, st);
    launch_check_finite(n * nrhs, x, fin, st);
    if (download(fin, 1, st)[0]) throw Error(LSDD_E_INVAL, "right-hand side or initial iterate has NaN/Inf");
    auto& B = h->pb[0];
    double* rr = h->sc;
    std::vector<lsdd_info> out((size_t)nrhs);
    bool breakdown = false;
    for (int32_t k = 0; k < nrhs && !breakdown; ++k) {
        const double* bk = b + (int64_t)k * n;
        double* xk = x + (int64_t)k * n;
        lsdd_info& f = out[k];
        f.setup_s = h->setup_s;
        // r = b - A x and its norm
        auto resid = [&] {
            traced(h, "pcg_spmv", full_apply_bytes(l0, 8.0, 8.0, true),
                   [&] { Cyc<double, 1>::spmv(l0, l0.d_val, xk, B.r, bk, st); });
            launch_seg_dot(h->seg, 1, B.r, B.r, nullptr, nullptr, h->part, rr, nullptr, st);
            const double v = std::sqrt(download(rr, 1, st)[0]);
            if (h->tr.on) h->tr.flush();
            return v;
        };
        const double r0 = resid();
        if (!std::isfinite(r0)) {
            breakdown = true;
            break;
        }
        if (r0 == 0.0) {
            f.converged = 1;
            continue;
        }
        double rel = 1.0;
        int32_t it = 0;
        while (it < h->prm.max_iter) {
            precond<1>(h, B.r, B.z);
            launch_axpy(n, 1.0, B.z, xk, st);
            ++it;
            rel = resid() / r0;
            if (!std::isfinite(rel)) {
                breakdown = true;
                break;
            }
            if (rel <= h->prm.rtol) break;
        }
        f.iters = it;
        f.rel_res = rel;
        f.converged = (!breakdown && rel <= h->prm.rtol) ? 1 : 0;
    }
    HIPCHK(hipGetLastError());
    sync(st);
    const double ts = now_s() - t0;
    bool allconv = true;
    for (auto& f : out) {
        f.solve_s = ts;
        allconv = allconv && f.converged;
    }
    if (info) std::copy(out.begin(), out.end(), info);
    if (breakdown) throw Error(LSDD_E_BREAKDOWN, "non-finite residual in the standalone cycle iteration");
    if (!allconv) {
        g_err = "the standalone cycle iteration did not reach rtol within max_iter";
        return LSDD_E_NOCONV;
    }
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_set_cycle_precision(lsdd_hierarchy* h, int32_t precision) {
    ABI_BEGIN
    if (!h || precision < 0 || precision > 2) throw Error(LSDD_E_INVAL, "bad argument");
    if (precision == 1 && h->prm.precision < 1)
        throw Error(LSDD_E_INVAL, "the FP32 cycle needs a hierarchy set up with precision >= 1");
    if (precision == 2 && h->prm.precision != 2)
        throw Error(LSDD_E_INVAL, "the mixed cycle needs a hierarchy set up with precision = 2");
    if (precision == 2 && h->prm.smoother != 0)
        throw Error(LSDD_E_UNSUPPORTED, "the mixed cycle runs the multiplicative Schwarz smoother only");
    h->cycle_prec = precision;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_set_solve_params(lsdd_hierarchy* h, double rtol, int32_t max_iter) {
    ABI_BEGIN
    if (!h || !(rtol > 0.0) || max_iter < 1) throw Error(LSDD_E_INVAL, "bad argument");
    h->prm.rtol = rtol;
    h->prm.max_iter = max_iter;
    reset_graphs(h);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_set_graph(lsdd_hierarchy* h, int32_t on) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    if (h->st) HIPCHK(hipStreamSynchronize(h->st));
    h->use_graph = on != 0;
    reset_graphs(h);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_segments(const lsdd_hierarchy* h, int32_t* n_seg, int64_t* seg_off) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    if (n_seg) *n_seg = h->seg.n_seg;
    if (seg_off) std::copy(h->seg_off.begin(), h->seg_off.end(), seg_off);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_autotune(lsdd_hierarchy* h, int32_t block, void* hip_stream) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    h->st = (hipStream_t)hip_stream;
    if (block) {
        if (!h->pb[1].B) {
            ensure_block_vectors(h);
            alloc_pcg(h, 1);
        }
        if (h->cycle_prec == 2) throw Error(LSDD_E_UNSUPPORTED, "the mixed cycle runs single right-hand sides only");
        if (h->cycle_prec == 1) autotune_levels<float, NRB>(h);
        else autotune_levels<double, NRB>(h);
    } else {
        if (h->cycle_prec >= 1) autotune_levels<float, 1>(h);
        else autotune_levels<double, 1>(h);
    }
    reset_graphs(h);
    HIPCHK(hipGetLastError());
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_set_level_tuning(lsdd_hierarchy* h, int32_t level, const int32_t* in) {
    ABI_BEGIN
    if (!h || !in || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    auto one_of = [](int32_t v, std::initializer_list<int32_t> ok) {
        return std::find(ok.begin(), ok.end(), v) != ok.end();
    };
    if (!one_of(in[0], {8, 16, 32, 64}) || !one_of(in[1], {4, 8, 16, 32, 64}) || !one_of(in[2], {2, 4, 8}) ||
        !one_of(in[3], {8, 32}) || !one_of(in[4], {0, 1}) || !one_of(in[5], {0, 1, 2, 3, 4}) || !one_of(in[6], {0, 1}))
        throw Error(LSDD_E_INVAL, "launch shape outside the autotuner's candidates");
    Level& lv = *h->L[level];
    if (in[5] && !lv.d_scoff)
        throw Error(LSDD_E_UNSUPPORTED, "shared column lists: the level's pattern is not supernode-blocked");
    if (in[5] >= 2 && !lv.d_rblk)
        throw Error(LSDD_E_UNSUPPORTED, "supernode row blocks: the level has no sweep row blocks");
    if (in[4] && !build_elem_apply(h, lv))
        throw Error(LSDD_E_UNSUPPORTED, "element apply: only on level 0 of a hierarchy built from element blocks "
                                        "of at most 128 DOFs");
    lv.eapply = in[4];
    lv.sup = in[5];
    lv.fact_stash = in[6];
    lv.lanes = in[0];
    lv.lanes_b = in[1];
    lv.fl = in[3];
    if (!lv.coarsest && in[2] != lv.chl) {
        set_chunk(h, lv, in[2]);
        sync(h->st);
    }
    reset_graphs(h);
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_level_tuning(const lsdd_hierarchy* h, int32_t level, int32_t* out) {
    ABI_BEGIN
    if (!h || !out || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    const Level& lv = *h->L[level];
    out[0] = lv.lanes;
    out[1] = lv.lanes_b;
    out[2] = lv.chl;
    out[3] = lv.fl;
    out[4] = lv.eapply;
    out[5] = lv.sup;
    out[6] = lv.fact_stash;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_level_segments(const lsdd_hierarchy* h, int32_t level, int64_t* inst_off, int32_t* terminal) {
    ABI_BEGIN
    if (!h || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    const Level& lv = *h->L[level];
    if (inst_off) std::copy(lv.inst_off.begin(), lv.inst_off.end(), inst_off);
    if (terminal) {
        std::fill(terminal, terminal + lv.inst_off.size() - 1, 0);
        for (int32_t i : lv.term) terminal[i] = 1;
    }
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_trace(lsdd_hierarchy* h, int32_t on) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    if (h->st) HIPCHK(hipStreamSynchronize(h->st));
    h->tr.flush();
    if (on) h->tr.agg.clear();
    h->tr.on = on != 0;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_trace_get(lsdd_hierarchy* h, int32_t idx, char* name, int32_t name_len, int64_t* launches,
                           double* ms, double* bytes) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    HIPCHK(hipStreamSynchronize(h->st));
    h->tr.flush();
    if (idx < 0 || idx >= (int32_t)h->tr.agg.size()) throw Error(LSDD_E_INVAL, "trace index out of range");
    const Trace::Agg& a = h->tr.agg[idx];
    if (name && name_len > 0) {
        std::strncpy(name, a.name.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = a.launches;
    if (ms) *ms = a.ms;
    if (bytes) *bytes = a.bytes;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_hierarchy_info(const lsdd_hierarchy* h, int32_t* levels, int64_t* n_l, int64_t* nnz_l, double* oc,
                                double* gc) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    const size_t L = h->L.size();
    if (levels) *levels = (int32_t)L;
    double sn = 0, snnz = 0;
    for (size_t l = 0; l < L; ++l) {
        if (n_l) n_l[l] = h->L[l]->n;
        if (nnz_l) nnz_l[l] = h->L[l]->nnz;
        sn += (double)h->L[l]->n;
        snnz += (double)h->L[l]->nnz;
    }
    if (oc) *oc = snnz / (double)h->L[0]->nnz;
    if (gc) *gc = sn / (double)h->L[0]->n;
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_level_sizes(const lsdd_hierarchy* h, int32_t level, int64_t* sizes) {
    ABI_BEGIN
    if (!h || !sizes || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    const Level& lv = *h->L[level];
    for (int i = 0; i < 8; ++i) sizes[i] = 0;
    sizes[0] = lv.n;
    sizes[1] = lv.nnz;
    sizes[7] = lv.el.count();
    if (!lv.coarsest) {
        sizes[2] = lv.cl.n_agg;
        sizes[3] = lv.zoff.empty() ? 0 : lv.zoff.back();
        sizes[4] = (int64_t)lv.cl.sub_dofs.size();
        sizes[5] = lv.n_colors;
        sizes[6] = lv.coff.empty() ? 0 : lv.coff.back();
    }
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_export_level(const lsdd_hierarchy* h, int32_t level, int32_t* agg_of_dof, int32_t* k, double* Z,
                              double* mu, int32_t* colors, int64_t* rowptr, int32_t* col, double* val,
                              int32_t* omega_sizes) {
    ABI_BEGIN
    if (!h || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    const Level& lv = *h->L[level];
    hipStream_t st = h->st;
    if (rowptr) std::copy(lv.pat.ptr.begin(), lv.pat.ptr.end(), rowptr);
    if (col) std::copy(lv.pat.idx.begin(), lv.pat.idx.end(), col);
    if (val) {
        HIPCHK(hipMemcpyAsync(val, lv.d_val, lv.nnz * sizeof(double), hipMemcpyDeviceToHost, st));
        sync(st);
    }
    if (lv.coarsest) return LSDD_OK;
    if (agg_of_dof) std::copy(lv.agg_of_dof.begin(), lv.agg_of_dof.end(), agg_of_dof);
    if (k) std::copy(lv.k.begin(), lv.k.end(), k);
    if (colors) std::copy(lv.colors.begin(), lv.colors.end(), colors);
    if (omega_sizes)
        for (int32_t i = 0; i < lv.cl.n_agg; ++i) omega_sizes[i] = (int32_t)(lv.cl.sub_ptr[i + 1] - lv.cl.sub_ptr[i]);
    if (Z && lv.zoff.back() > 0) {
        HIPCHK(hipMemcpyAsync(Z, lv.d_Z, lv.zoff.back() * sizeof(double), hipMemcpyDeviceToHost, st));
        sync(st);
    }
    if (mu) {
        HIPCHK(hipMemcpyAsync(mu, lv.d_mu, lv.n * sizeof(double), hipMemcpyDeviceToHost, st));
        sync(st);
    }
    return LSDD_OK;
    ABI_END
}

namespace lsdd {
// Gram factors of the grouped element blocks of a coarse level (Sec. 5.1: a sum
// of SPSD element blocks is SPSD and so has a Gram factor of its own, which may
// replace the rows G P inherited from the finer level; factorisation of
// Sec. 5.2).  Every block is factored with diagonal pivoting (largest remaining
// diagonal entry, lowest index among equal ones), truncated when that entry is
// at most n_g eps max diag; the rows come out in the original index order.  The
// blocks are SPSD only up to the rounding of the Galerkin products, so no SPSD
// test is applied.  Runs once per level, on the first request.
void coarse_gram(lsdd_hierarchy* h, Level& lv) {
    Arena& ar = h->arena;
    hipStream_t st = h->st;
    const int64_t ne = lv.el.count();
    const int64_t tot = lv.blk_off[ne];
    constexpr int64_t CH = 65535;                       // views per batched launch
    double* W = ar.alloc<double>(std::max<int64_t>(tot, 1));
    int32_t* d_perm = ar.alloc<int32_t>(std::max<int64_t>(lv.el.ptr[ne], 1));
    int32_t* d_rank = ar.alloc<int32_t>(std::max<int64_t>(ne, 1));
    double* d_maxd = ar.alloc<double>(CH);
    double* d_tol = ar.alloc<double>(CH);
    double* G = ar.alloc<double>(std::max<int64_t>(tot, 1));
    if (tot) HIPCHK(hipMemcpyAsync(W, lv.d_blocks, tot * sizeof(double), hipMemcpyDeviceToDevice, st));
    Batched bt;
    bt.st = st;
    bt.alloc = [](void* c, size_t b) { return static_cast<Arena*>(c)->get(b); };
    bt.release = [](void* c, void* p) { static_cast<Arena*>(c)->release(p); };
    bt.ctx = &ar;
    std::vector<int32_t> ranks(ne, 0);
    for (int64_t e0 = 0; e0 < ne; e0 += CH) {
        const int64_t cnt = std::min(CH, ne - e0);
        std::vector<View> v(cnt);
        std::vector<int32_t> lead(cnt, 0), rank;
        for (int64_t i = 0; i < cnt; ++i) {
            const int32_t n = (int32_t)(lv.el.ptr[e0 + i + 1] - lv.el.ptr[e0 + i]);
            v[i] = View{lv.blk_off[e0 + i], n, n, n, 0};
        }
        launch_views_max_diag((int32_t)cnt, W, bt.put(0, v), d_maxd, st);
        std::vector<double> maxd = download(d_maxd, cnt, st), tol(cnt);
        for (int64_t i = 0; i < cnt; ++i) tol[i] = v[i].rows * DBL_EPSILON * std::max(maxd[i], 0.0);
        HIPCHK(hipMemcpyAsync(d_tol, tol.data(), cnt * sizeof(double), hipMemcpyHostToDevice, st));
        bt.pstrf_trailing(W, v, lead, d_tol, rank, d_perm + lv.el.ptr[e0]);      // synchronises
        std::copy(rank.begin(), rank.end(), ranks.begin() + e0);
        HIPCHK(hipMemcpyAsync(d_rank + e0, rank.data(), cnt * sizeof(int32_t), hipMemcpyHostToDevice, st));
        launch_gram_rows(cnt, lv.d_elem_ptr + e0, lv.d_blk_off + e0, W, d_perm + lv.el.ptr[e0], d_rank + e0, G, st);
        HIPCHK(hipGetLastError());
        sync(st);
    }
    bt.free_all();
    for (void* p : {(void*)W, (void*)d_perm, (void*)d_rank, (void*)d_maxd, (void*)d_tol}) ar.release(p);
    lv.d_G = G;
    lv.ranks = std::move(ranks);
}
}  // namespace lsdd

lsdd_status lsdd_export_gram_level(lsdd_hierarchy* h, int32_t level, int64_t* elem_ptr, int32_t* elem_dofs,
                                   int32_t* ranks, double* G) {
    ABI_BEGIN
    if (!h || level < 0 || level >= (int32_t)h->L.size()) throw Error(LSDD_E_INVAL, "bad argument");
    Level& lv = *h->L[level];
    if (elem_ptr) std::copy(lv.el.ptr.begin(), lv.el.ptr.end(), elem_ptr);
    if (elem_dofs) std::copy(lv.el.dofs.begin(), lv.el.dofs.end(), elem_dofs);
    if (ranks || G) {
        if (!lv.d_G) coarse_gram(h, lv);
        if (ranks) std::copy(lv.ranks.begin(), lv.ranks.end(), ranks);
        if (G) {
            HIPCHK(hipMemcpyAsync(G, lv.d_G, lv.blk_off.back() * sizeof(double), hipMemcpyDeviceToHost, h->st));
            sync(h->st);
        }
    }
    return LSDD_OK;
    ABI_END
}

lsdd_status lsdd_export_gram(const lsdd_hierarchy* h, int32_t* ranks, double* G) {
    ABI_BEGIN
    if (!h) throw Error(LSDD_E_INVAL, "NULL hierarchy");
    const Level& l0 = *h->L[0];
    if (ranks) std::copy(l0.ranks.begin(), l0.ranks.end(), ranks);
    if (G) {
        HIPCHK(hipMemcpyAsync(G, l0.d_G, l0.blk_off.back() * sizeof(double), hipMemcpyDeviceToHost, h->st));
        sync(h->st);
    }
    return LSDD_OK;
    ABI_END
}

}  // extern "C"
