// Internal interface between the host runtime and the KSG kernels.
//
// A launch processes a list of jobs.  A job is a set of estimates of
// I(X;Y|Z) that share the rows of Y and Z and differ only in the permutation
// applied to the rows of X (the candidate's own estimate uses the identity,
// its surrogates the keyed shuffles).  Different jobs of one launch may have
// different N, column counts and k.
//
// Work is split into items (job, estimate group, query tile, reference split)
// pulled from one atomic counter by a persistent grid:
//   phase A: fused items (whole reference range: k-NN pass, then the count
//            pass, then the digamma partial sums) for jobs with one split, and
//            k-NN items (partial top-k over one reference range) for jobs with
//            several splits;
//   phase B: count items for jobs with several splits; they wait until the
//            last k-NN item of their (job, group, tile) has merged the radii.
// All phase-A items are handed out before any phase-B item, and waits only go
// from phase B to phase A, so every wait ends.
#pragma once

#include <cstdint>

namespace mte {

constexpr int kMaxCols = 64;       // dx + dy + dz per job
constexpr int kMaxDx = 16;
constexpr int kMaxDy = 8;
constexpr int kMaxDz = 31;
constexpr int kMaxK = 16;
constexpr int kBlock = 256;        // threads per block (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = 64;         // rows per fixed-order partial sum

// One estimate's surrogate key (identity when `ident` != 0).
struct EstKey {
    uint64_t h;        // key hash of (seed, cand, s)
    uint32_t ident;
    uint32_t pad;
};

struct Job {
    const float *cols[kMaxCols];  // X columns, then Y, then Z; each N floats
    int n, dx, dy, dz, k;
    int n_est;                    // estimates
    int rs;                       // reference splits (1 = fused items)
    int split_len;                // references per split (multiple of 64)
    int n_tiles;                  // query tiles of the launch's tile size
    int n_groups;                 // estimate groups of the launch's group size
    int64_t a_off, b_off;         // first item index in phase A and phase B
    const EstKey *keys;           // [n_est]
    float *xp;                    // [n_est][dx][n] permuted X (scratch)
    double *chunk;                // partial sums per 64-row chunk (scratch): [n_est][ceil(n/64)],
                                  // list path [ceil(n/64)][n_est]
    float *part;                  // [rs][n_est][n][KMAX] partial top-k (rs > 1)
    float *eps;                   // [n_est][n] radii (rs > 1, or diagnostics)
    int32_t *cnt;                 // [rs][n_est][3][n] per-split counts (rs > 1)
    uint32_t *sync;               // counters, see SyncLayout
    double *out;                  // [n_est] results
    float *diag_eps;              // optional [n_est][n]
    int32_t *diag_cnt;            // optional [n_est][3][n] (n_xz, n_yz, n_z)
    // neighbour-list path only (see ListSet): list set index, and the
    // permuted X columns transposed so that the estimates of one row are
    // adjacent: xt[c][i][e] = X_c[pi_e(i)] ([dx][n][n_est]) for the scan (xp
    // holds the same values estimate-major for the fallback).  The per-row
    // counts go to pk; eps and cnt are the caller's diagnostics ([n_est][n],
    // [n_est][3][n]) or null.
    int set;
    float *xt;
    int theiler;                  // Theiler window w: pairs with |i - j| <= w are left out
    int reps;                     // replications R (rows: R blocks of n/R, replication-major)
    int rep_shuffle;              // surrogates shuffle the replication order (else rows within each)
    // list path without Z (dz = 0, dx = 1): the job's X column sorted
    // ascending (n floats), for the n_x range counts; null otherwise
    float *xs;
    // list path: each (row, estimate)'s counts in one word,
    // n_xz | n_yz << kPackBits | n_z << 2 kPackBits ([n_est][n])
    uint64_t *pk;
    // list path with one Z column (rank counts, see ListSet::zs): the set's
    // rank of each row, the permuted X in rank order, estimate-major
    // (xr[e][c][r] = X_c[pi_e(zord[r])], [n_est][dx][n]), and each pair's
    // radius from the k-NN scan (er[e][i], -1 for a pair left to the
    // all-rows redo); null otherwise
    const int32_t *zrank;
    float *xr;
    float *er;
};

// Counts of the list path are packed kPackBits to a field: N <= kListMaxN.
constexpr int kPackBits = 21;
constexpr int kListMaxN = 1 << kPackBits;

// Largest N of a list-path job without Z (its X column is sorted in LDS).
constexpr int kNoZSortMax = 16384;

// Neighbour lists of one (Y, Z) sample, shared by every job of a launch whose
// Y and Z columns are the same.  For row i, list 1 holds the other rows j with
// the (Y,Z) max-norm distance d_yz(i,j) in the smallest key buckets that fit
// m1 entries, list 2 the same for the Z distance d_z(i,j) and m2.  A key is
// the top 12 bits of the distance's float encoding (8 exponent and 4
// mantissa bits), so a list is ordered by bucket, not fully sorted.  List 2 entries
// also carry d_yz (d_yz >= d_z, so every row with d_yz below a radius is in
// the part of list 2 below that radius).  bound[i][w] is a
// lower bound of every unlisted distance (+inf when nothing is left out), so
// a radius r <= bound[i][w] is decided by the list alone.
struct LEnt {
    float d;                      // d_yz
    int32_t j;                    // row
};

struct LEnt2 {
    float dz;                     // d_z (the list key)
    float dyz;                    // d_yz, so that n_yz is counted from this list too
    int32_t j;                    // row
};

constexpr int kListPad = 8;                   // sentinel entries after each row's list

struct ListSet {
    const float *cols[kMaxDy + kMaxDz];   // Y columns, then Z columns
    float *zy;                    // [dz + dy][n] contiguous copy: Z columns, then Y (build input)
    int32_t *order;               // [n] the scan's row order in launches of several jobs: rows
                                  // grouped by Morton cell of their Z, Y coordinates; null: identity
    int n, dy, dz;
    int theiler;                  // Theiler window of the rows (|i - j| <= w left out)
    int m1, m2;                   // list capacities per row
    int s1, s2;                   // row strides: capacity + kListPad sentinels
    LEnt *l1;                     // [n][s1]  (Y,Z) list
    LEnt2 *l2;                    // [n][s2]  Z list
    int32_t *len;                 // [n][2]
    float *bound;                 // [n][2]
    // One Z column and n <= kRankMaxN: the rows sorted by z, so that the rows
    // within a radius of a row's z are one range of ranks (float subtraction
    // is monotone in its first operand).  zs[r] the r-th smallest z, zord[r]
    // its row, zrank the inverse, yr[c][r] = Y_c[zord[r]].  The counts of
    // such a set's jobs come from these ranges, not from the Z list (whose
    // capacity is then kRankListCap).  Null otherwise.
    float *zs;
    int32_t *zord;
    int32_t *zrank;
    float *yr;
};

constexpr int kCoopLanes = 4;                 // default cooperative-finish threshold of the scan
constexpr int kRankMaxN = 32768;              // rank counts: rows ranked by O(n^2) compares
constexpr int kRankListCap = 8;               // Z-list capacity of a set counted by ranks

constexpr int kBuildRows = 2;                // rows per build block when N <= 2^16
constexpr int kLeanRows = 2;                 // rows per block of the compiled-dimension build
// Compiled-dimension build: dz <= kBuildFixedDz Z columns and one Y column.
constexpr int kBuildFixedDz = 12;
constexpr int kXcds = 8;   // accelerator complex dies (one L2 each) of an MI355X
constexpr int kBuildCopies = 1;              // histogram copies per row (spread LDS atomics)
constexpr int kListStatWord = 16;
constexpr int kListStatSlots = 64;            // spread so that the atomics do not queue on one address
constexpr int kListStatStride = 16;           // words (64 bytes) per slot
constexpr int kListCounterWords = kListStatWord + kListStatSlots * kListStatStride;
constexpr int kKeyShift = 19;                 // 4096 key buckets
constexpr int kKeyBins = 1 << (32 - kKeyShift - 1);

// One launch of the list path over `n_jobs` jobs (all with dz > 0).
struct ListLaunch {
    const Job *jobs;              // device
    const ListSet *sets;          // device
    const int64_t *lane_off;      // [n_jobs+1] prefix sums of n * n_est
    const int64_t *row_off;       // [n_sets+1] prefix sums of the sets' n
    const int64_t *build_off;     // [n_sets+1] prefix sums of the build blocks per set
    int64_t build_blocks;
    int build_qb;                 // rows per build block: kBuildRows (N <= 2^16) or 1
    int build_pack;               // 16-bit packed histograms (every set has N <= 2^16)
    int build_dz;                 // > 0: every set has this many Z columns and one Y column
                                  // (the build's compiled-dimension forms)
    int build_kind;               // 0 generic dimensions (list_build_kernel); 1 compiled
                                  // dimensions (list_build_dz_kernel)
    int stats;                    // non-zero: the scan accumulates its entry counts
    const int64_t *est_off;       // [n_jobs+1] prefix sums of n_est
    int n_jobs, n_sets;
    int64_t lanes, rows, ests;
    uint64_t *failq;              // [lanes] (job << 40 | i * n_est + e) of undecided pairs
    uint32_t *counters;           // [0] undecided pairs; from word kListStatWord,
                                  // kListStatSlots slots of kListStatStride words each
                                  // holding two uint64 totals of list entries read (k-NN
                                  // scan, Z-list scan); kListCounterWords words, zeroed
                                  // per launch
    int kmax, dxm;                // compile-time classes of the scan kernel
    int fb_grid;                  // blocks of the fallback kernel
    int max_chunks;               // largest ceil(n / kChunk) of the jobs (reduction grid)
    int sortx;                    // some job has no Z: sort the X columns (Job::xs)
    int coop_lanes;               // the scan finishes cooperatively once this many lanes remain
    int grouped;                  // 1 (one job): lanes over 64-estimate groups, XCD-contiguous
                                  // blocks; 2 (several jobs): XCD-dealt units, below
    // grouped == 2: unit u = (job, 64-estimate group of the job, the last one
    // taking the remainder), its lanes row-major in the set's row order and
    // padded to whole blocks, runs on XCD u % kXcds.  xcd_off[x * (unit_t + 1)
    // + t] is the first block, counting XCD x's blocks alone, of x's t-th unit
    // (unit x + t * kXcds; the entry at t = unit_t, and past x's last unit,
    // is x's block count); unit_info[u] = job << 32 | group.
    const int64_t *xcd_off;
    const int64_t *unit_info;
    int unit_t, n_units;
    int64_t scan_blocks;          // grid of the scan
    int scan_step;                // list entries per step of the scan's lane-by-lane loops (4, 8)
    int rank_sets;                // sets counted by ranks (ListSet::zs)
    int64_t rank_waves;           // rank-count waves: sum over those sets' jobs of
                                  // n_est * ceil(n / 64)
    const int64_t *rank_off;      // [n_jobs+1] prefix sums of each job's rank-count waves
    int max_rank_n;               // largest n of a set counted by ranks
};

// Counter words of one job (all zero before a launch):
//   [0, G*T)        k-NN items done per (group, tile)
//   [G*T, 2*G*T)    radii ready per (group, tile)
//   [2GT, 3GT)      count items done per (group, tile)
//   [3GT, 3GT+G)    tiles finished per group
inline int64_t sync_words(int n_groups, int n_tiles) {
    return 3LL * n_groups * n_tiles + n_groups;
}

// Tile configurations compiled into the library.
struct TileCfg {
    int kmax;   // top-k register slots (k <= kmax)
    int g;      // estimates per lane
    int qp;     // queries per lane
    int dzm;    // Z column capacity
    int dym;    // Y column capacity
    int dxm;    // X column capacity
};

struct LaunchInfo {
    int64_t items_a, items_b;     // item counts of the two phases
    int grid;                     // persistent blocks
};

// Compiled configurations of the all-pairs kernel for jobs with few estimates
// (solo.hip): top-k capacity, Z, Y and X column capacities, estimates and
// query rows per wave.
struct SoloCfg {
    int kmax, dzm, dym, dxm, g, qp;
    int fz;                                  // >= 0: compiled dimensions (dz = fz, dy = dx = 1)
};
constexpr int kSoloMaxEstimates = 7;         // jobs with more take the persistent kernel
int solo_variant_count();
bool solo_variant(int i, SoloCfg *cfg);
// One wave per (job, estimate group, query tile); wave_off: [n_jobs+1] prefix
// sums of each job's waves.  Writes Job::pk (and the diagnostics).
int launch_solo(int variant, const Job *jobs_dev, int n_jobs, const int64_t *wave_off, int64_t total_waves,
                void *stream);

// Host-side launch helpers implemented in kernels.hip.
// jobs_dev: device copy of `n_jobs` Job records; work: 2 device words
// (queue head, error flag) cleared by `launch_reset`.
int kernel_variant_count();
bool kernel_variant(int i, TileCfg *cfg);
int variant_blocks_per_cu(int variant);
int launch_reset(uint32_t *words, int64_t n_words, void *stream);
// Permuted X columns: total_blocks work items (blk_off: [n_jobs+1] prefix
// sums of each job's items), on a grid of at most max_grid blocks (0: one
// block per item) that take the items in turn.
int launch_permute(const Job *jobs_dev, int n_jobs, int64_t total_blocks, const int64_t *blk_off,
                   void *stream, int64_t max_grid = 0);
int launch_main(int variant, const Job *jobs_dev, int n_jobs, const int64_t *a_off_dev,
                const int64_t *b_off_dev, const LaunchInfo &li, uint32_t *work,
                const double *harm, void *stream);

int launch_list_zy(const ListLaunch &L, void *stream);      // the sets' contiguous Y,Z copies; clears the counters
int launch_list_order(const ListLaunch &L, void *stream);  // the scan's row order (several jobs)
int launch_list_build(const ListLaunch &L, void *stream);
int launch_list_sortx(const ListLaunch &L, void *stream);
int launch_list_scan(const ListLaunch &L, void *stream);
int launch_list_rank_sort(const ListLaunch &L, void *stream);   // ranks of the one-Z-column sets
int launch_list_rank_count(const ListLaunch &L, void *stream);  // their jobs' counts
int launch_list_fallback(const ListLaunch &L, void *stream);
int launch_list_reduce(const ListLaunch &L, const double *harm, void *stream);

// Host reference of the surrogate permutation (same definition as the device).
uint64_t mix64(uint64_t z);
uint64_t surrogate_key(uint64_t seed, uint32_t cand, uint32_t s);
void permutation_host(uint64_t h, int64_t n, uint32_t *out);
// Source rows of one surrogate over R replications of n/R rows (the device's
// definition; R = 1 without rep_shuffle is permutation_host).
void replication_source_rows_host(uint64_t h, int64_t n, int reps, int rep_shuffle, uint32_t *out);
// MTE_SHUFFLE_REPLICATIONS when R! >= S, else MTE_SHUFFLE_WITHIN.
int shuffle_mode(int reps, int S);
// Blocks of the permute kernel for one estimate of a job.
inline int64_t permute_blocks(int64_t n, int reps) { return (int64_t)reps * ((n / reps + 1023) / 1024); }

}  // namespace mte
