// Scratch layout of the symmetric subdomain product (host and device).
//
// A subdomain of size m has nt = ceil(m / 64) tile rows.  Work item (I, ch)
// covers tiles J = ch * chl .. min(ch * chl + chl, I + 1) - 1 of tile row I and
// writes one 64-entry row part; every tile strictly below the diagonal also
// yields one 64-entry column part.  Row parts come first, ordered by (I, ch);
// column parts follow, ordered by (I, J) with J < I.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsdd {

constexpr int SUB_MAX_CHUNK = 8;   // largest number of tiles per work item

// number of row parts of tile rows 0 .. I-1: sum_{i < I} ceil((i + 1) / chl)
__host__ __device__ inline int64_t symv_rowpart_off(int I, int chl) {
    int64_t full = I / chl, rem = I % chl;
    return chl * full * (full + 1) / 2 + rem * (full + 1);
}

// scratch entries of one subdomain with nt tile rows
__host__ __device__ inline int64_t symv_scratch_len(int nt, int chl) {
    return (symv_rowpart_off(nt, chl) + (int64_t)nt * (nt - 1) / 2) * 64;
}

}  // namespace lsdd
