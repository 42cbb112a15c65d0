// Host integer setup (see graph.hpp).  Sec. 2 of the paper: aggregates
// (eq. agg_def), row-touching sets and overlaps (eqs. calR_def, overlap_def),
// multiplicities (eq. row_multiplicity); Sec. 6: standard aggregation passes.
#include "graph.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace lsdd {

namespace {

// Build a CSR from (row, col) pairs, deduplicated and sorted per row.
Csr pairs_to_csr(int64_t nrows, std::vector<std::pair<int32_t, int32_t>>& pr) {
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    Csr c;
    c.ptr.assign(nrows + 1, 0);
    c.idx.resize(pr.size());
    for (size_t t = 0; t < pr.size(); ++t) {
        c.ptr[pr[t].first + 1]++;
        c.idx[t] = pr[t].second;
    }
    for (int64_t r = 0; r < nrows; ++r) c.ptr[r + 1] += c.ptr[r];
    return c;
}

// Transpose of an incidence list: for each target, the sources listing it.
Csr transpose(int64_t n_targets, const std::vector<int64_t>& ptr, const std::vector<int32_t>& idx) {
    Csr t;
    t.ptr.assign(n_targets + 1, 0);
    for (int32_t v : idx) t.ptr[v + 1]++;
    for (int64_t r = 0; r < n_targets; ++r) t.ptr[r + 1] += t.ptr[r];
    t.idx.resize(idx.size());
    std::vector<int64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
    int64_t nsrc = (int64_t)ptr.size() - 1;
    for (int64_t s = 0; s < nsrc; ++s)
        for (int64_t q = ptr[s]; q < ptr[s + 1]; ++q) t.idx[fill[idx[q]]++] = (int32_t)s;
    return t;
}

}  // namespace

Csr supernode_graph(int32_t n_super, const std::vector<int32_t>& node_of_dof, const ElemList& el) {
    // element -> distinct supernodes, then supernode -> elements, then neighbours
    std::vector<int64_t> eptr(el.count() + 1, 0);
    std::vector<int32_t> enodes;
    enodes.reserve(el.dofs.size());
    for (int64_t e = 0; e < el.count(); ++e) {
        size_t start = enodes.size();
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) enodes.push_back(node_of_dof[el.dofs[q]]);
        std::sort(enodes.begin() + start, enodes.end());
        enodes.erase(std::unique(enodes.begin() + start, enodes.end()), enodes.end());
        eptr[e + 1] = (int64_t)enodes.size();
    }
    Csr n2e = transpose(n_super, eptr, enodes);
    Csr g;
    g.ptr.assign(n_super + 1, 0);
    std::vector<int32_t> mark(n_super, -1);
    for (int32_t s = 0; s < n_super; ++s) {
        mark[s] = s;
        size_t start = g.idx.size();
        for (int64_t q = n2e.ptr[s]; q < n2e.ptr[s + 1]; ++q) {
            int32_t e = n2e.idx[q];
            for (int64_t r = eptr[e]; r < eptr[e + 1]; ++r) {
                int32_t t = enodes[r];
                if (mark[t] != s) {
                    mark[t] = s;
                    g.idx.push_back(t);
                }
            }
        }
        std::sort(g.idx.begin() + start, g.idx.end());
        g.ptr[s + 1] = (int64_t)g.idx.size();
    }
    return g;
}

std::vector<int32_t> standard_aggregation(const Csr& g, int32_t* n_agg) {
    const int64_t n = g.rows();
    std::vector<int32_t> agg(n, -1);
    int32_t na = 0;
    // roots: the whole neighbourhood is still free
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int64_t q = g.ptr[i]; q < g.ptr[i + 1] && free_nb; ++q) free_nb = agg[g.idx[q]] < 0;
        if (!free_nb) continue;
        agg[i] = na;
        for (int64_t q = g.ptr[i]; q < g.ptr[i + 1]; ++q) agg[g.idx[q]] = na;
        ++na;
    }
    // attach: lowest-index neighbour that was aggregated in the root phase
    std::vector<int32_t> root_phase(agg);
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        int32_t best = -1;
        for (int64_t q = g.ptr[i]; q < g.ptr[i + 1]; ++q) {
            int32_t j = g.idx[q];
            if (root_phase[j] >= 0 && (best < 0 || j < best)) best = j;
        }
        if (best >= 0) agg[i] = root_phase[best];
    }
    // leftovers
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        agg[i] = na;
        for (int64_t q = g.ptr[i]; q < g.ptr[i + 1]; ++q)
            if (agg[g.idx[q]] < 0) agg[g.idx[q]] = na;
        ++na;
    }
    *n_agg = na;
    return agg;
}

std::vector<int32_t> aggregate(const Csr& g0, int passes, int32_t* n_agg) {
    const int64_t n = g0.rows();
    std::vector<int32_t> agg(n);
    for (int64_t i = 0; i < n; ++i) agg[i] = (int32_t)i;
    int32_t na = (int32_t)n;
    Csr g = g0;
    for (int p = 0; p < passes; ++p) {
        int32_t nn = 0;
        std::vector<int32_t> a = standard_aggregation(g, &nn);
        for (int64_t i = 0; i < n; ++i) agg[i] = a[agg[i]];
        // quotient graph on the new aggregates
        std::vector<std::pair<int32_t, int32_t>> pr;
        for (int64_t u = 0; u < g.rows(); ++u)
            for (int64_t q = g.ptr[u]; q < g.ptr[u + 1]; ++q) {
                int32_t au = a[u], av = a[g.idx[q]];
                if (au != av) pr.emplace_back(au, av);
            }
        g = pairs_to_csr(nn, pr);
        na = nn;
    }
    *n_agg = na;
    return agg;
}

Closure build_closure(int64_t n, const std::vector<int32_t>& agg_of_dof, int32_t n_agg, const ElemList& el) {
    Closure c;
    c.n_agg = n_agg;
    // aggregates (ascending DOFs)
    c.agg_ptr.assign(n_agg + 1, 0);
    for (int64_t d = 0; d < n; ++d)
        if (agg_of_dof[d] >= 0) c.agg_ptr[agg_of_dof[d] + 1]++;
    for (int32_t i = 0; i < n_agg; ++i) c.agg_ptr[i + 1] += c.agg_ptr[i];
    c.agg_dofs.resize(c.agg_ptr[n_agg]);
    c.pos_in_agg.assign(n, -1);
    {
        std::vector<int64_t> fill(c.agg_ptr.begin(), c.agg_ptr.end() - 1);
        for (int64_t d = 0; d < n; ++d) {
            int32_t i = agg_of_dof[d];
            if (i < 0) continue;
            c.pos_in_agg[d] = (int32_t)(fill[i] - c.agg_ptr[i]);
            c.agg_dofs[fill[i]++] = (int32_t)d;
        }
    }
    // element -> touched aggregates; multiplicity; aggregate -> touching elements
    const int64_t ne = el.count();
    c.mult.assign(ne, 0);
    std::vector<int64_t> tptr(ne + 1, 0);
    std::vector<int32_t> touched;
    for (int64_t e = 0; e < ne; ++e) {
        size_t start = touched.size();
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q)
            if (agg_of_dof[el.dofs[q]] >= 0) touched.push_back(agg_of_dof[el.dofs[q]]);
        std::sort(touched.begin() + start, touched.end());
        touched.erase(std::unique(touched.begin() + start, touched.end()), touched.end());
        tptr[e + 1] = (int64_t)touched.size();
        c.mult[e] = (int32_t)(tptr[e + 1] - tptr[e]);
        c.max_mult = std::max(c.max_mult, c.mult[e]);
    }
    Csr a2e = transpose(n_agg, tptr, touched);
    c.cl_ptr = a2e.ptr;
    c.cl_elems = a2e.idx;
    // overlaps: omega first, then the rest of the closure ascending
    c.sub_ptr.assign(n_agg + 1, 0);
    std::vector<int32_t> mark(n, -1);
    std::vector<int32_t> gam;
    for (int32_t i = 0; i < n_agg; ++i) {
        for (int64_t q = c.agg_ptr[i]; q < c.agg_ptr[i + 1]; ++q) {
            c.sub_dofs.push_back(c.agg_dofs[q]);
            mark[c.agg_dofs[q]] = i;
        }
        gam.clear();
        for (int64_t q = c.cl_ptr[i]; q < c.cl_ptr[i + 1]; ++q) {
            int32_t e = c.cl_elems[q];
            for (int64_t r = el.ptr[e]; r < el.ptr[e + 1]; ++r) {
                int32_t d = el.dofs[r];
                if (mark[d] != i) {
                    mark[d] = i;
                    gam.push_back(d);
                }
            }
        }
        std::sort(gam.begin(), gam.end());
        c.sub_dofs.insert(c.sub_dofs.end(), gam.begin(), gam.end());
        c.sub_ptr[i + 1] = (int64_t)c.sub_dofs.size();
    }
    return c;
}

void a_closure_overlaps(const Csr& pat, const std::vector<double>& val, double tol, Closure& c) {
    const int64_t n = pat.rows();
    std::vector<double> diag(n, 0.0);
    for (int64_t p = 0; p < n; ++p)
        for (int64_t q = pat.ptr[p]; q < pat.ptr[p + 1]; ++q)
            if (pat.idx[q] == p) diag[p] = val[q];
    std::vector<int64_t> ptr(c.n_agg + 1, 0);
    std::vector<int32_t> dofs;
    dofs.reserve(c.sub_dofs.size());
    std::vector<int32_t> mark(n, -1), gam;
    for (int32_t i = 0; i < c.n_agg; ++i) {
        for (int64_t q = c.agg_ptr[i]; q < c.agg_ptr[i + 1]; ++q) mark[c.agg_dofs[q]] = i;
        gam.clear();
        for (int64_t q = c.agg_ptr[i]; q < c.agg_ptr[i + 1]; ++q) {
            const int32_t r = c.agg_dofs[q];
            dofs.push_back(r);
            for (int64_t t = pat.ptr[r]; t < pat.ptr[r + 1]; ++t) {
                const int32_t p = pat.idx[t];
                if (mark[p] == i) continue;
                if (std::fabs(val[t]) > tol * std::sqrt(std::fabs(diag[p] * diag[r]))) {
                    mark[p] = i;
                    gam.push_back(p);
                }
            }
        }
        std::sort(gam.begin(), gam.end());
        dofs.insert(dofs.end(), gam.begin(), gam.end());
        ptr[i + 1] = (int64_t)dofs.size();
    }
    c.sub_ptr = std::move(ptr);
    c.sub_dofs = std::move(dofs);
}

std::vector<int32_t> color_subdomains(int64_t n, const Closure& c, const ElemList& el, int32_t* n_colors) {
    const int32_t na = c.n_agg;
    Csr d2s = transpose(n, c.sub_ptr, c.sub_dofs);        // DOF -> subdomains containing it
    // S_e: the subdomains an element meets (sorted, distinct); every pair in one S_e conflicts
    Csr es;
    es.ptr.assign(el.count() + 1, 0);
    std::vector<int32_t> subs;
    for (int64_t e = 0; e < el.count(); ++e) {
        subs.clear();
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) {
            int32_t d = el.dofs[q];
            for (int64_t r = d2s.ptr[d]; r < d2s.ptr[d + 1]; ++r) subs.push_back(d2s.idx[r]);
        }
        std::sort(subs.begin(), subs.end());
        subs.erase(std::unique(subs.begin(), subs.end()), subs.end());
        es.idx.insert(es.idx.end(), subs.begin(), subs.end());
        es.ptr[e + 1] = (int64_t)es.idx.size();
    }
    Csr se = transpose(na, es.ptr, es.idx);              // subdomain -> elements meeting it
    // greedy in ascending index: the smallest colour that no already coloured
    // conflicting subdomain holds (stamped per subdomain, no conflict list stored)
    std::vector<int32_t> color(na, -1), stamp;
    int32_t nc = 0;
    for (int32_t i = 0; i < na; ++i) {
        for (int64_t q = se.ptr[i]; q < se.ptr[i + 1]; ++q) {
            const int32_t e = se.idx[q];
            for (int64_t r = es.ptr[e]; r < es.ptr[e + 1]; ++r) {
                const int32_t k = es.idx[r];
                if (k < i) stamp[color[k]] = i;
            }
        }
        int32_t col = 0;
        while (col < nc && stamp[col] == i) ++col;
        color[i] = col;
        if (col == nc) {
            ++nc;
            stamp.push_back(-1);
        }
    }
    *n_colors = nc;
    return color;
}

Csr assembled_pattern(int64_t n, const ElemList& el) {
    Csr d2e = transpose(n, el.ptr, el.dofs);
    Csr p;
    p.ptr.assign(n + 1, 0);
    std::vector<int64_t> mark(n, -1);
    for (int64_t d = 0; d < n; ++d) {
        size_t start = p.idx.size();
        for (int64_t q = d2e.ptr[d]; q < d2e.ptr[d + 1]; ++q) {
            int32_t e = d2e.idx[q];
            for (int64_t r = el.ptr[e]; r < el.ptr[e + 1]; ++r) {
                int32_t t = el.dofs[r];
                if (mark[t] != d) {
                    mark[t] = d;
                    p.idx.push_back(t);
                }
            }
        }
        std::sort(p.idx.begin() + start, p.idx.end());
        p.ptr[d + 1] = (int64_t)p.idx.size();
    }
    return p;
}

bool assembled_pattern_blocked(int64_t n, const ElemList& el, const std::vector<int32_t>& node_of_dof,
                               int32_t n_super, Csr& p) {
    std::vector<int64_t> first(n_super + 1, -1);
    for (int64_t d = 0; d < n; ++d) {
        const int32_t s = node_of_dof[d];
        if (d > 0 && s < node_of_dof[d - 1]) return false;
        if (first[s] < 0) first[s] = d;
    }
    first[n_super] = n;
    for (int32_t s = n_super - 1; s >= 0; --s)
        if (first[s] < 0) first[s] = first[s + 1];
    // supernodes of every element (each once) and the elements of every supernode
    ElemList es;
    es.ptr.assign(1, 0);
    std::vector<int32_t> last(n_super, -1);
    std::vector<int64_t> cnt(n_super, 0);
    for (int64_t e = 0; e < el.count(); ++e) {
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) {
            const int32_t s = node_of_dof[el.dofs[q]];
            if (last[s] != (int32_t)e) {
                last[s] = (int32_t)e;
                cnt[s] = 0;
                es.dofs.push_back(s);
            }
            ++cnt[s];
        }
        // every element must hold whole supernodes (distinct DOFs per element)
        for (int64_t r = es.ptr.back(); r < (int64_t)es.dofs.size(); ++r) {
            const int32_t s = es.dofs[r];
            if (cnt[s] != first[s + 1] - first[s]) return false;
        }
        es.ptr.push_back((int64_t)es.dofs.size());
    }
    Csr s2e = transpose(n_super, es.ptr, es.dofs);
    // supernode neighbourhoods, sorted
    Csr nb;
    nb.ptr.assign(n_super + 1, 0);
    std::vector<int32_t> mark(n_super, -1);
    for (int32_t s = 0; s < n_super; ++s) {
        const size_t start = nb.idx.size();
        for (int64_t q = s2e.ptr[s]; q < s2e.ptr[s + 1]; ++q) {
            const int32_t e = s2e.idx[q];
            for (int64_t r = es.ptr[e]; r < es.ptr[e + 1]; ++r) {
                const int32_t t = es.dofs[r];
                if (mark[t] != s) {
                    mark[t] = s;
                    nb.idx.push_back(t);
                }
            }
        }
        std::sort(nb.idx.begin() + start, nb.idx.end());
        nb.ptr[s + 1] = (int64_t)nb.idx.size();
    }
    // expand: every DOF of s gets the DOF ranges of its neighbours, ascending
    std::vector<int64_t> rowlen(n_super, 0);
    for (int32_t s = 0; s < n_super; ++s)
        for (int64_t q = nb.ptr[s]; q < nb.ptr[s + 1]; ++q) rowlen[s] += first[nb.idx[q] + 1] - first[nb.idx[q]];
    p.ptr.assign(n + 1, 0);
    for (int64_t d = 0; d < n; ++d) p.ptr[d + 1] = p.ptr[d] + rowlen[node_of_dof[d]];
    p.idx.resize(p.ptr[n]);
    for (int64_t d = 0; d < n; ++d) {
        const int32_t s = node_of_dof[d];
        int64_t o = p.ptr[d];
        for (int64_t q = nb.ptr[s]; q < nb.ptr[s + 1]; ++q)
            for (int64_t c = first[nb.idx[q]]; c < first[nb.idx[q] + 1]; ++c) p.idx[o++] = (int32_t)c;
    }
    return true;
}

CoarseGroups group_coarse(const ElemList& el, const std::vector<int32_t>& agg_of_dof,
                          const std::vector<int32_t>& k, const std::vector<int64_t>& coarse_off) {
    CoarseGroups cg;
    const int32_t na = (int32_t)k.size();
    std::vector<int32_t> compact(na, -1);
    int32_t ns = 0;
    for (int32_t i = 0; i < na; ++i)
        if (k[i] > 0) compact[i] = ns++;
    cg.n_super = ns;
    cg.node_of_cdof.resize(coarse_off[na]);
    for (int32_t i = 0; i < na; ++i)
        for (int64_t d = coarse_off[i]; d < coarse_off[i + 1]; ++d) cg.node_of_cdof[d] = compact[i];
    // Groups keyed by the sorted set of aggregates (with k > 0) an element touches, numbered
    // in order of first occurrence.  Open-addressing table of group ids; the keys live
    // once per group in a flat array.
    const int64_t ne = el.count();
    int64_t cap = 64;
    while (cap < 2 * ne + 64) cap <<= 1;
    std::vector<int32_t> table(cap, -1);
    std::vector<uint64_t> ghash;
    std::vector<int64_t> kptr(1, 0);
    std::vector<int32_t> kval, gid(ne, -1), t;
    auto hash_of = [](const std::vector<int32_t>& v) {
        uint64_t h = 1469598103934665603ull;                   // FNV-1a over the entries
        for (int32_t x : v) {
            h ^= (uint64_t)(uint32_t)x;
            h *= 1099511628211ull;
        }
        return h;
    };
    for (int64_t e = 0; e < ne; ++e) {
        t.clear();
        for (int64_t q = el.ptr[e]; q < el.ptr[e + 1]; ++q) {
            int32_t a = agg_of_dof[el.dofs[q]];
            if (a >= 0 && k[a] > 0) t.push_back(a);
        }
        std::sort(t.begin(), t.end());
        t.erase(std::unique(t.begin(), t.end()), t.end());
        if (t.empty()) continue;
        const uint64_t h = hash_of(t);
        int64_t slot = (int64_t)(h & (uint64_t)(cap - 1));
        int32_t g = -1;
        while (table[slot] >= 0) {
            const int32_t c = table[slot];
            if (ghash[c] == h && kptr[c + 1] - kptr[c] == (int64_t)t.size() &&
                std::equal(t.begin(), t.end(), kval.begin() + kptr[c])) {
                g = c;
                break;
            }
            slot = (slot + 1) & (cap - 1);
        }
        if (g < 0) {
            g = (int32_t)ghash.size();
            table[slot] = g;
            ghash.push_back(h);
            kval.insert(kval.end(), t.begin(), t.end());
            kptr.push_back((int64_t)kval.size());
        }
        gid[e] = g;
    }
    const int32_t ng = (int32_t)ghash.size();
    cg.coarse.ptr.assign(ng + 1, 0);
    for (int32_t g = 0; g < ng; ++g) {
        for (int64_t q = kptr[g]; q < kptr[g + 1]; ++q)
            for (int64_t d = coarse_off[kval[q]]; d < coarse_off[kval[q] + 1]; ++d)
                cg.coarse.dofs.push_back((int32_t)d);
        cg.coarse.ptr[g + 1] = (int64_t)cg.coarse.dofs.size();
    }
    cg.mem_ptr.assign(ng + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
        if (gid[e] >= 0) ++cg.mem_ptr[gid[e] + 1];
    for (int32_t g = 0; g < ng; ++g) cg.mem_ptr[g + 1] += cg.mem_ptr[g];
    cg.mem_elems.resize(cg.mem_ptr[ng]);
    std::vector<int64_t> fill(cg.mem_ptr.begin(), cg.mem_ptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
        if (gid[e] >= 0) cg.mem_elems[fill[gid[e]]++] = (int32_t)e;
    return cg;
}

}  // namespace lsdd
