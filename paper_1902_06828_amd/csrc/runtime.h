// Host runtime shared by the C ABI, the greedy driver and the request loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "mte.h"

namespace mte {

// ---------------------------------------------------------------- errors
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
#define MTE_HIP(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return ::mte::hip_fail(e_, #expr); \
    } while (0)

// ---------------------------------------------------------------- memory
// Caching device allocator.  Freed blocks are kept and a request takes the
// smallest cached block that holds it, if that block is at most a quarter
// (plus 64 MiB) larger; otherwise a new block.  Batches of the request loop
// differ in size from one to the next, so reuse by exact size alone would
// allocate nearly every batch anew and fill the device with cached blocks
// until a failed allocation freed them all (hipFree waits for the device).
// in_use counts the blocks' real sizes.
class DeviceAllocator {
public:
    void *alloc(size_t bytes);          // nullptr on failure
    void release(void *p, size_t bytes);
    void trim();                        // free every cached block
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    size_t cached() const { return cached_; }
    void reset_peak() { peak_ = in_use_; }
private:
    void free_cached_locked();
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live_;     // block sizes of the blocks handed out
    size_t in_use_ = 0, peak_ = 0, cached_ = 0;
    size_t cache_cap_ = 0;              // cached bytes kept at most (set on first release)
};

// RAII device buffer from the context allocator.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    int ensure(size_t n);               // MTE_OK or MTE_ENOMEM
    void reset();
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Pinned host staging buffer.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf();
    int ensure(size_t n);
    void reset();
};

// ---------------------------------------------------------------- jobs
// Host description of one job (device pointers for the columns and outputs).
struct JobSpec {
    const float *cols[kMaxCols] = {};
    int n = 0, dx = 0, dy = 0, dz = 0, k = 0;
    int theiler = 0;                   // Theiler window w (|i - j| <= w left out)
    int reps = 1;                      // replications: rows are reps blocks of n/reps rows
    int rep_shuffle = 0;               // surrogates shuffle the replication order
    std::vector<EstKey> keys;          // one per estimate
    double *out = nullptr;             // device [n_est]
    float *diag_eps = nullptr;         // device [n_est][n] or null
    int32_t *diag_cnt = nullptr;       // device [n_est][3][n] or null
    int n_est() const { return (int)keys.size(); }
};

// Launch choices that change no result: the all-pairs kernel's tile
// configuration and split count, and the list path's knobs (0 = default).
struct TileChoice {
    int variant = -1;
    int rs_mult = 1;                   // multiplier on the heuristic split count
    int build_qb = 0;                  // rows per block of the compiled-dimension build (2 or 4)
    int coop_lanes = 0;                // the scan's cooperative-finish threshold
    int grouped = -1;                  // one-job launches: estimate-group lane order (1) or not (0)
    int scan_step = 0;                 // the scan's entries per step (4, 8)
    int perm_cu = 0;                   // blocks per CU of the permutation beside the build (0: default)
};

// Which path runs each job of a batch: -1 = all-pairs kernel, otherwise the
// index of the job's neighbour-list set (jobs with the same N and the same Y
// and Z columns share one set).  The list path is used for jobs whose set
// carries at least kListMinEstimates estimates, that have Z columns or else
// one X column and N <= kNoZSortMax, and whose permuted X columns hold fewer
// than 2^31 values; the
// environment variable MTE_FORCE_MODE=brute|list overrides that (results are
// the same either way).
constexpr int kListMinEstimates = 8;
int assign_paths(const std::vector<JobSpec> &specs, std::vector<int> *set_of, int *n_sets);
// Of the jobs that do not take the list path: those with at most
// kSoloMaxEstimates estimates and N <= kListMaxN take the few-estimate
// all-pairs kernel (solo.hip), the others the persistent kernel.
// MTE_FORCE_MODE=brute sends every such job to the persistent kernel,
// MTE_FORCE_MODE=solo every one the few-estimate kernel fits.
bool takes_solo(const JobSpec &sp);

// Timed stages (HIP events around each launch when timing is enabled).
enum Stage { kStageAllPairs = 0, kStageBuild, kStageScan, kStageFallback, kStageReduce, kStagePermute,
             kStageGaussGram, kStageGaussCmi, kStages };

// One launch: its tables, scratch and (optionally) a captured graph.
class Batch {
public:
    ~Batch();
    // Lay out and upload everything for `specs` with the given tile choice
    // (the tile choice only concerns the jobs of the all-pairs kernel).  With
    // `measure` set, only compute the device bytes the launch would hold
    // (device_bytes() after a real prepare) and allocate nothing.
    int prepare(const std::vector<JobSpec> &specs, const TileChoice &tc, hipStream_t s,
                size_t *measure = nullptr);
    // Enqueue the launch sequence on s (graph replay if captured).
    int enqueue(hipStream_t s, bool use_graph);
    // Non-zero when a kernel reported an error (reads device words; syncs s).
    int check_error(hipStream_t s);
    // Launches of the autotuner: direct, no stage timing, no list statistics.
    int enqueue_quiet(hipStream_t s);
    size_t device_bytes() const;
    int variant() const { return variant_; }
    int64_t estimates() const { return n_est_total_; }
private:
    int capture();
    int launch_direct(hipStream_t s);
    int launch_all(hipStream_t s, bool timed);
    int prepare_pairs(const std::vector<JobSpec> &specs, const TileChoice &tc, hipStream_t s, size_t *measure);
    int prepare_lists(const std::vector<JobSpec> &specs, const std::vector<int> &set_of, int n_sets,
                      const TileChoice &tc, hipStream_t s, size_t *measure);
    int prepare_solo(const std::vector<JobSpec> &specs, hipStream_t s, size_t *measure);
    // few-estimate part (solo kernel, then the list path's reduction)
    int n_sjobs_ = 0, svariant_ = -1;
    Job *sjobs_dev_ = nullptr;
    int64_t *s_wave_off_ = nullptr, *s_blk_off_ = nullptr;
    int64_t s_total_waves_ = 0, s_permute_blocks_ = 0;
    ListLaunch sl_{};
    DevBuf stables_, sscratch_;
    // neighbour-list part
    int n_ljobs_ = 0;
    ListLaunch ll_{};
    int64_t lpermute_blocks_ = 0;
    Job *ljobs_dev_ = nullptr;
    int64_t *lblk_off_ = nullptr;
    DevBuf ltables_, lscratch_, lcounters_;
    int64_t n_est_pairs_ = 0;
    // all-pairs part
    int variant_ = -1;
    int n_jobs_ = 0;
    int64_t n_est_total_ = 0;
    LaunchInfo li_{};
    int64_t permute_blocks_ = 0;
    int64_t sync_total_ = 0;           // words, including the 2 work words
    DevBuf tables_, scratch_, sync_;
    Job *jobs_dev_ = nullptr;
    int64_t *a_off_ = nullptr, *b_off_ = nullptr, *blk_off_ = nullptr;
    uint32_t *work_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    bool graph_failed_ = false;
    bool quiet_ = false;                // a tuning launch: leaves the statistics alone
    // fork/join of the list part's permutation onto the side stream
    hipEvent_t fork_ = nullptr, join_ = nullptr;
    int perm_cu_ = 0;                   // the permutation's blocks per CU beside the build (0: uncapped)
};

// ---------------------------------------------------------------- context
struct Ctx {
    std::mutex mu;
    bool inited = false;
    int device = -1;
    int n_cu = 0;
    size_t budget = 0;
    hipStream_t capture_stream = nullptr;
    hipStream_t side_stream = nullptr;   // work that runs beside a launch's main stream
    DeviceAllocator alloc;
    // harmonic numbers H[0..harm_n]; old tables stay alive until shutdown
    double *harm = nullptr;
    int64_t harm_n = 0;
    std::vector<double *> retired;
    // autotuner: shape key -> choice ("P..." keys: all-pairs tiles of a
    // batch; "L..." keys: list-path knobs of a job shape), the choices made
    // or loaded (for mte_tune_report), the device's architecture and the
    // file the choices persist in ("" = none)
    std::map<std::string, TileChoice> tuned;
    struct TuneNote {
        std::string key;
        TileChoice tc;
        double ms;
        int from_disk;
    };
    std::vector<TuneNote> tune_log;
    std::string arch, tune_file;
    // kernel timing per stage
    bool timing = false;
    // a is shared with the previous pair's b (and not returned or destroyed
    // twice) when own_a is false
    struct Pending { int stage; hipEvent_t a, b; bool own_a; };
    std::vector<Pending> pending_events;
    std::vector<hipEvent_t> event_pool;   // read timing events, for reuse
    int64_t timed_launches[kStages] = {};
    double timed_ms[kStages] = {};
    // list path statistics (from checked launches)
    int64_t list_pairs = 0, list_undecided = 0;
    int64_t list_seen[2] = {};
    bool list_stats = false;           // scan kernels count the list entries they read
};

Ctx &ctx();
// A timing event: from the pool of read ones, else a new one.
int timing_event(hipEvent_t *e);
int ensure_init();                     // lazily initialises device 0
int ensure_harm(int64_t n);            // H table covers 0..n
const double *harm_table();

// Pick the tile variant classes for a set of jobs; -1 if nothing fits.
int variant_for(const std::vector<JobSpec> &specs, int g_pref);
// Choose the launch choices of a batch: a choice tuned before for its shape
// (in this process or read from the tuning file) or, on a shape's first
// call, by the autotuner as `mode` allows:
//   kTuneNone   look up only (the request loop: tuning launches would hold
//               memory outside its budget)
//   kTuneBatch  time the candidates on the batch itself (device calls)
//   kTuneShape  time the list knobs on a one-job launch of the batch's first
//               list job (host calls, greedy rounds); only for batches of at
//               least kTuneMinPairs (row, estimate) pairs
// MTE_TUNE=0 turns tuning off (heuristic choices).
enum { kTuneNone = 0, kTuneBatch = 1, kTuneShape = 2 };
constexpr int64_t kTuneMinPairs = int64_t(1) << 20;
int choose_tiles(const std::vector<JobSpec> &specs, hipStream_t s, int mode, TileChoice *out);

// The tile choice for jobs run on the all-pairs kernel whatever path
// assign_paths would give them: the autotuner's cached choice for the shape
// when there is one, else the heuristic.  Allocates nothing.
int pair_tiles(const std::vector<JobSpec> &specs, TileChoice *out);

// Layout of the all-pairs part of a launch: the Job records (scratch,
// counter and key pointers not yet set), the work-item and permute-block
// offsets, each job's byte offsets within one scratch region and its first
// counter word, and the sizes of the tables (jobs, keys, three offset
// arrays, each rounded to 256 bytes).
struct PairPlan {
    std::vector<Job> jobs;
    std::vector<int64_t> a_off, b_off, blk_off;
    struct Off {
        size_t xp = 0, chunk = 0, part = 0, eps = 0, cnt = 0;
        int64_t sync = 0;
    };
    std::vector<Off> offs;
    size_t scratch_bytes = 0;
    int64_t sync_words = 0;           // including the 2 work words
    int64_t n_keys = 0;
    LaunchInfo li{};
    int64_t permute_blocks = 0;
    size_t tbl_jobs = 0, tbl_keys = 0, tbl_offs = 0;
};
int plan_pairs(const std::vector<JobSpec> &specs, const TileChoice &tc, PairPlan *plan);
// Point every job's scratch, counters and keys into the given regions.
void bind_pairs(PairPlan &plan, uint8_t *scratch, uint32_t *sync, EstKey *keys_dev);

// Address of the allocation-free call's static scratch array on `device`
// (bound once per device at initialisation; see noalloc.hip).
int noalloc_bind(int device);

// Run a batch to completion on an internal stream (used by the host-pointer
// calls and the greedy driver).  Outputs land in the JobSpec device buffers.
int run_blocking(const std::vector<JobSpec> &specs, hipStream_t s);

// Validation shared by the entry points.
int validate_dims(int dx, int dy, int dz, int64_t n, int k);
int validate_host_finite(const float *p, int64_t count, const char *name);
int validate_theiler(int64_t n, int k, int theiler);
int autocorr_decay_time(const float *x, int64_t T, int max_lag);

// Host mirror of the device harmonic table (same summation order).
double harmonic_host(int64_t n);

void record_timing_pair(int stage, hipEvent_t a, hipEvent_t b, bool own_a = true);
// several pairs at once (one launch's: a readout then sees all of them or none,
// so an event shared by two of them is never returned to the pool early)
void record_timing_pairs(const std::vector<Ctx::Pending> &pairs);

// Per-node z-score of a host series [R][P][T] (see runtime.cpp).
void standardise_host(const float *in, int R, int P, int64_t T, float *out);

}  // namespace mte
