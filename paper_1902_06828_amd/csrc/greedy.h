// Greedy source selection over resident columns (shared by the single-target
// entry points and network inference).
#pragma once

#include <cstdint>

#include "runtime.h"

namespace mte {

// Device columns of the embedded variables: lag-shifted windows of a
// resident [P][T] series, or, with R replications, rows of an embedding
// buffer [P][l_m+1][N] gathered from a resident [R][P][T] series (the rows of
// replication r at r*n_r.., n_r = T - l_m).
struct Columns {
    const float *series = nullptr;
    int64_t T = 0;
    int l_m = 0;
    const float *emb = nullptr;
    int64_t N = 0;
    int reps = 1;
    const float *col(int node, int lag) const {
        return emb ? emb + ((size_t)node * (l_m + 1) + lag) * (size_t)N : series + (size_t)node * T + (l_m - lag);
    }
};

int select_sources_columns(const Columns &c, int target, const int32_t *candidates, int n_candidates,
                           int max_lag_sources, double alpha, const mte_opts &o, mte_result *out);
int resident_columns(const float *data, int P, int64_t T, int l_m, int R, hipStream_t s, DevBuf *series,
                     DevBuf *emb, Columns *c);
int greedy_check(int P, int64_t T, int target, const int32_t *cands, int n_cands, int l_s, double alpha,
                 const mte_opts &o, mte_result *out);
mte_opts greedy_opts(const mte_opts *o);

}  // namespace mte
