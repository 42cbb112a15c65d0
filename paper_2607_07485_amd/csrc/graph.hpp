// Host-side integer setup of one LS-AMG-DD level: the aggregation graph,
// standard aggregation, G-row closures, multiplicities, subdomain colouring,
// CSR patterns and the grouping of coarse element rows.  Pure C++ (no HIP).
#pragma once
#include <cstdint>
#include <vector>

namespace lsdd {

// Compressed adjacency / incidence lists (ptr has size+1 entries).
struct Csr {
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    int64_t rows() const { return (int64_t)ptr.size() - 1; }
};

// Elements of one level: element e has support dofs[ptr[e] .. ptr[e+1]).
struct ElemList {
    std::vector<int64_t> ptr;
    std::vector<int32_t> dofs;
    int64_t count() const { return (int64_t)ptr.size() - 1; }
};

// Supernodes s ~ t iff some element holds DOFs of both (all connections strong).
Csr supernode_graph(int32_t n_super, const std::vector<int32_t>& node_of_dof, const ElemList& el);

// Standard aggregation on an undirected graph (no self loops): roots with a
// fully free neighbourhood in ascending order, then every free node joins the
// root-phase aggregate of its lowest-index aggregated neighbour, then leftovers
// group with their free neighbours.  Returns the aggregate of every node.
std::vector<int32_t> standard_aggregation(const Csr& g, int32_t* n_agg);

// `passes` rounds of standard aggregation, each on the quotient graph of the last.
std::vector<int32_t> aggregate(const Csr& g, int passes, int32_t* n_agg);

// Overlapping subdomains of one level.
struct Closure {
    int32_t n_agg = 0;
    std::vector<int64_t> agg_ptr;   // omega_i = agg_dofs[agg_ptr[i] .. agg_ptr[i+1]) ascending
    std::vector<int32_t> agg_dofs;
    std::vector<int32_t> pos_in_agg;    // per DOF: its index inside its aggregate (-1: none)
    std::vector<int64_t> sub_ptr;   // Omega_i: omega_i ascending, then Gamma_i ascending
    std::vector<int32_t> sub_dofs;
    std::vector<int64_t> cl_ptr;    // elements with a DOF in omega_i, ascending
    std::vector<int32_t> cl_elems;
    std::vector<int32_t> mult;      // per element: number of aggregates it touches
    int32_t max_mult = 0;
};

// DOFs with agg_of_dof < 0 belong to no aggregate (problem instances whose
// hierarchy ended on this level); elements made of such DOFs touch no aggregate.
Closure build_closure(int64_t n, const std::vector<int32_t>& agg_of_dof, int32_t n_agg, const ElemList& el);

// Replace the overlaps of c by algebraic A-closures (Def. "algebraic A-closure"):
// Omega_i = omega_i, then the DOFs p outside omega_i with
// |A(p,q)| > tol sqrt(|A(p,p) A(q,q)|) for some q in omega_i, ascending.  A is the
// level's symmetric operator (CSR with pattern pat, values val).  Every such p
// shares an element with omega_i, so the new overlap is a subset of the G-row one.
void a_closure_overlaps(const Csr& pat, const std::vector<double>& val, double tol, Closure& c);

// Greedy colouring of subdomains: i and k conflict iff an element meets both
// Omega_i and Omega_k.  Ascending index, smallest free colour.
std::vector<int32_t> color_subdomains(int64_t n, const Closure& c, const ElemList& el, int32_t* n_colors);

// Structural CSR pattern of sum_e R_e^T 1 R_e (sorted columns).
Csr assembled_pattern(int64_t n, const ElemList& el);

// The same pattern when the DOFs of every supernode form a contiguous range
// (node_of_dof non-decreasing) and every element holds whole supernodes (always
// on the coarse levels, often on level 0): computed on supernodes and expanded
// by ranges (rows of one supernode share their columns).  Returns false (p
// untouched) if either property fails.
bool assembled_pattern_blocked(int64_t n, const ElemList& el, const std::vector<int32_t>& node_of_dof,
                               int32_t n_super, Csr& p);

// Coarse element rows: elements touching the same set of aggregates with k > 0
// share their coarse support and multiplicity; they are grouped into one coarse
// element whose block is the sum of theirs.
struct CoarseGroups {
    ElemList coarse;                 // coarse supports (coarse DOF numbering)
    std::vector<int64_t> mem_ptr;    // members of group g: mem_elems[mem_ptr[g] .. mem_ptr[g+1])
    std::vector<int32_t> mem_elems;
    std::vector<int32_t> node_of_cdof;   // coarse supernode = compact index of the parent aggregate
    int32_t n_super = 0;
};

CoarseGroups group_coarse(const ElemList& el, const std::vector<int32_t>& agg_of_dof,
                          const std::vector<int32_t>& k, const std::vector<int64_t>& coarse_off);

}  // namespace lsdd
