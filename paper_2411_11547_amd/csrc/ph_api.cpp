// Host runtime and C ABI of libpairhmm (include/ph.h).
//
// A plan is built once per problem shape: it validates the batch structure
// and lengths, assigns every read length to a kernel configuration (lanes P
// per pair, rows K per lane; the paper's (p, k) template grid, Section
// III-B/III-C), counts the pairs of every length bin, and allocates the
// device scratch.  A forward call then enqueues, on the caller's stream:
//   1. (explicit-parameter mode) exponentiation of the log10 parameters;
//   2. on-device binning: histogram, scan and scatter of the pairs by
//      (length bin, haplotype length), Section III-A stage 3 / Section III-C;
//   3. one persistent FP32 sweep per non-empty bin, longest bin first, as
//      parallel branches (Section III-C runs one kernel per index list on its
//      own stream);
//   4. the FP64 sweep over the pairs whose FP32 sum fell below the rescue
//      threshold, one persistent launch per read-length class.
// The whole sequence is captured once into a HIP graph and replayed while
// the problem and output pointers stay the same.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ph.h"
#include "ph_internal.h"

using namespace ph;

namespace {

thread_local std::string g_err;

ph_status fail(ph_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace

namespace ph {
// the calling thread's message for ph_last_error(), set by other host sources
void set_last_error(const char *msg) { g_err = msg ? msg : ""; }
}  // namespace ph

namespace {

#define HIPCHK(x)                                                                           \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) return fail(PH_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// One bin of the FP32 sweep: reads up to max_m bases in groups of P lanes x
// K rows.  A table line may add a haplotype-length split "n_split P2 K2":
// pairs of that read range whose haplotype has at least n_split bases go to
// a second bin of P2 x K2 (a table entry that follows its parent, with the
// same max_m, so that the read-length map never selects it).
struct TuneEntry {
    int max_m, P, K;
    int n_split = 0, P2 = 0, K2 = 0;
};

// haplotype-length bucket of the binning key (16-column buckets below 1024,
// 128-column buckets above; the kernels' pair_key uses the same)
int hap_bucket(int64_t n) { return n < 1024 ? (int)(n >> 4) : 64 + (int)std::min<int64_t>((n - 1024) >> 7, 63); }

constexpr int kSideStreams = 4;
constexpr int kStageEvents = 5;

std::once_flag g_lut_once;
hipError_t g_lut_status = hipSuccess;
std::once_flag g_lut_adj_once;
hipError_t g_lut_adj_status = hipSuccess;

// adjoint checkpoint workspaces: the grid of a launch shrinks to fit
constexpr int64_t kAdjWsFloats = (int64_t)1 << 30;    // 4 GiB, FP32 pass
constexpr int64_t kAdjWs64Doubles = (int64_t)1 << 28;  // 2 GiB, FP64 pass

int rescue_class_of(int m) { return m < 128 ? 0 : m < 256 ? 1 : m < 512 ? 2 : 3; }

// The library's own bin table, shortest reads first: 16 lanes x K rows
// (K = 1..16) up to 255 bases, then 64 lanes x K rows (K = 5..16).  Written
// into a fixed array (the allocation-free forward uses it too); returns the
// number of entries.
int builtin_table(TuneEntry *t)
{
    int n = 0;
    for (int K = 1; K <= 16; ++K) t[n++] = {16 * K - 1, 16, K};
    for (int K = 5; K <= 16; ++K) t[n++] = {64 * K - 1, 64, K};
    return n;
}

std::vector<TuneEntry> default_table(int force_p)
{
    std::vector<TuneEntry> t;
    if (force_p) {
        for (int K = 1; K <= 16; ++K)
            if (fwd32_supported(force_p, K) && force_p * K - 1 <= kMaxReadLen)
                t.push_back({force_p * K - 1, force_p, K});
        return t;
    }
    TuneEntry b[kMaxBins];
    const int nb = builtin_table(b);
    t.assign(b, b + nb);
    return t;
}

// Table for the single-launch sweep: reads shorter than 48 share the K = 3 bin.
std::vector<TuneEntry> single_table()
{
    std::vector<TuneEntry> t;
    for (int K = 3; K <= 16; ++K) t.push_back({16 * K - 1, 16, K});
    for (int K = 5; K <= 16; ++K) t.push_back({64 * K - 1, 64, K});
    return t;
}

ph_status read_table(const char *path, std::vector<TuneEntry> &t)
{
    std::ifstream f(path);
    if (!f) return fail(PH_ERR_INVALID, "cannot open tune table %s", path);
    std::string line;
    t.clear();
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        const std::string body = line.substr(0, line.find('#'));
        std::istringstream ss(body);
        TuneEntry e;
        if (!(ss >> e.max_m >> e.P >> e.K)) return fail(PH_ERR_INVALID, "bad tune line: %s", line.c_str());
        if (!fwd32_supported(e.P, e.K)) return fail(PH_ERR_UNSUPPORTED, "tune entry P=%d K=%d not compiled", e.P, e.K);
        if (e.max_m > e.P * e.K - 1 || e.max_m < 1)
            return fail(PH_ERR_INVALID, "tune entry max_m=%d exceeds P*K-1 for P=%d K=%d", e.max_m, e.P, e.K);
        if (ss >> e.n_split) {
            if (!(ss >> e.P2 >> e.K2) || e.n_split < 1)
                return fail(PH_ERR_INVALID, "bad haplotype-length split in tune line: %s", line.c_str());
            if (!fwd32_supported(e.P2, e.K2))
                return fail(PH_ERR_UNSUPPORTED, "tune entry P=%d K=%d not compiled", e.P2, e.K2);
            if (e.max_m > e.P2 * e.K2 - 1)
                return fail(PH_ERR_INVALID, "tune entry max_m=%d exceeds P*K-1 for P=%d K=%d", e.max_m, e.P2, e.K2);
            const bool edge = e.n_split < 1024 ? e.n_split % 16 == 0
                                               : (e.n_split - 1024) % 128 == 0 && e.n_split <= 1024 + 63 * 128;
            if (!edge)
                return fail(PH_ERR_INVALID, "haplotype-length split %d is not a bucket edge (a multiple of 16 "
                            "below 1024, 1024 + a multiple of 128 up to 9088)", e.n_split);
        }
        t.push_back(e);
    }
    std::sort(t.begin(), t.end(), [](const TuneEntry &a, const TuneEntry &b) { return a.max_m < b.max_m; });
    if (t.empty()) return fail(PH_ERR_INVALID, "empty tune table %s", path);
    // neighbouring ranges with the same configuration form one bin
    std::vector<TuneEntry> merged;
    for (const TuneEntry &e : t) {
        const TuneEntry *b = merged.empty() ? nullptr : &merged.back();
        if (b && b->P == e.P && b->K == e.K && b->n_split == e.n_split && b->P2 == e.P2 && b->K2 == e.K2)
            merged.back().max_m = e.max_m;
        else
            merged.push_back(e);
    }
    // each split adds its second bin right after its parent
    t.clear();
    for (const TuneEntry &e : merged) {
        t.push_back(e);
        if (e.n_split) {
            TuneEntry a;
            a.max_m = e.max_m;
            a.P = e.P2;
            a.K = e.K2;
            t.push_back(a);
        }
    }
    if ((int)t.size() > kMaxBins - 1)
        return fail(PH_ERR_INVALID, "tune table has more than %d distinct bins", kMaxBins - 1);
    return PH_OK;
}

}  // namespace

struct ph_plan {
    int device = 0;
    int cus = 0;
    ph_plan_opts opts{};
    double threshold = 1e-28;
    int32_t nb = 0, nr = 0, nh = 0;
    int64_t P = 0, cells = 0, nread_bases = 0, nhap_bases = 0;
    int32_t max_m = 0, max_n = 0;

    std::vector<TuneEntry> table;      // bin b = table[table.size()-1-b] (longest first)
    std::vector<int> bin_grid;         // persistent grid per bin (0 = empty)
    int64_t class_pairs[kRescueClasses] = {0, 0, 0, 0};
    int rescue_grid[2][kRescueClasses] = {};  // [rescaled FP64, plain FP64] per class
    int plain_K = 0, plain_grid = 0;
    // reads longer than kMaxReadLen: one extra bin swept in windows
    int long_bin = -1, windows = 0, long_grid = 0, long64_grid = 0;
    int64_t long_pairs = 0, bnd_stride = 0;
    float *d_bnd32 = nullptr;
    double *d_bnd64 = nullptr;
    int32_t *d_long_rescue = nullptr;
    int split_at = -1;     // offset of the haplotype-length split table in d_m2bin (-1: none)
    std::vector<std::pair<int, int>> launch_order;  // FP32 stage: (bin, side stream) in launch order
    bool single = false;   // one persistent FP32 launch over all bins
    int single_grid = 0;
    // binned mode: work lists built from the shape at plan creation, with
    // chain tiles; the call copies the book image and writes the chain codes
    std::vector<int64_t> bin_tiles;    // tiles per bin
    int32_t chain_rec_base = 0;        // records of the lists; FP64 records of chain pairs follow
    bool chain_tiles = false;
    Book *d_book_img = nullptr;
    uint8_t *d_chain_codes = nullptr;

    int64_t *d_out_offset = nullptr;
    int16_t *d_m2bin = nullptr;
    int32_t *d_bin_G = nullptr;
    int32_t *d_hist = nullptr;
    PairRec *d_recs = nullptr;
    Book *d_book = nullptr;
    int32_t *d_bad = nullptr;          // ph_validate: count of base codes above 4
    int32_t *d_rescue = nullptr;
    double *d_lin = nullptr;
    int64_t lin_cap = 0;

    hipStream_t cap = nullptr;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, join[kSideStreams] = {};
    hipEvent_t ev[kStageEvents] = {};
    bool stages_recorded = false;

    // stage graphs of the forward ([0]) and of the Viterbi score ([1])
    hipGraph_t graph[2][3] = {};
    hipGraphExec_t exec[2][3] = {};
    std::vector<const void *> graph_key[2];

    hipStream_t last_stream = nullptr;
    bool forward_done = false;

    // host copy of the shape (adjoint tables are built from it on demand)
    std::vector<int32_t> h_rb, h_hb;
    std::vector<int64_t> h_ro, h_ho, h_out_off;

    // adjoint: records grouped by (P, K) configuration, tiled G = 64/P at a
    // time; one persistent launch per configuration, each workgroup with its
    // own checkpoint slice
    struct AdjRun {
        int P, K;
        int64_t rec_begin;
        int32_t nrec, ntiles, hs_bytes, grid;
        int64_t ws_stride;  // floats per workgroup
    };
    bool adj_built = false;
    ph_status adj_status = PH_OK;
    std::string adj_error;
    std::vector<AdjRun> adj_runs;
    AdjRec *d_adj_recs = nullptr;
    float *d_ws = nullptr;
    // gradients of reads with several pairs: per-pair rows, then a
    // fixed-order sum per read (no float atomics)
    float *d_grad_pair = nullptr;
    AdjRedRead *d_red = nullptr;
    int32_t n_red = 0;
    bool adj_zero = false;  // some read has no pair: its rows are zeroed
    int32_t *d_adj_ctr = nullptr;  // [2][kAdj64Classes] FP64 queue lengths, cursors; then one cursor per run
    // FP64 pass over the pairs the FP32 pass leaves out: queues per class,
    // [2][kAdj64Classes] counters (lengths, cursors), per-workgroup checkpoints
    int32_t *d_q64 = nullptr;
    double *d_ws64 = nullptr;
    int64_t q64_stride = 0, ws64_stride = 0;
    int32_t grid64 = 0, hs_bytes64 = 0;
    bool class64[kAdj64Classes] = {};
    hipEvent_t ev_adj[2] = {};
    bool adj_recorded = false;
    hipGraph_t adj_graph = nullptr;
    hipGraphExec_t adj_exec = nullptr;
    std::vector<const void *> adj_graph_key;
};

namespace {

void free_plan(ph_plan *p)
{
    if (!p) return;
    for (int v = 0; v < 2; ++v)
        for (int i = 0; i < 3; ++i) {
            if (p->exec[v][i]) (void)hipGraphExecDestroy(p->exec[v][i]);
            if (p->graph[v][i]) (void)hipGraphDestroy(p->graph[v][i]);
        }
    if (p->adj_exec) (void)hipGraphExecDestroy(p->adj_exec);
    if (p->adj_graph) (void)hipGraphDestroy(p->adj_graph);
    void *bufs[] = {p->d_out_offset, p->d_m2bin, p->d_bin_G, p->d_hist, p->d_recs, p->d_book, p->d_bad, p->d_rescue, p->d_lin,
                    p->d_book_img, p->d_chain_codes,
                    p->d_bnd32, p->d_bnd64, p->d_long_rescue,
                    p->d_adj_recs, p->d_ws, p->d_adj_ctr, p->d_q64, p->d_ws64, p->d_grad_pair, p->d_red};
    for (auto &e : p->ev_adj)
        if (e) (void)hipEventDestroy(e);
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : p->join)
        if (e) (void)hipEventDestroy(e);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (auto &s : p->side)
        if (s) (void)hipStreamDestroy(s);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
}

template <typename T>
ph_status dalloc(T **ptr, size_t count)
{
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)ptr, bytes);
    if (e != hipSuccess) return fail(PH_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return PH_OK;
}

ph_status check_problem(const ph_plan *p, const ph_problem *pb)
{
    if (!pb) return fail(PH_ERR_INVALID, "problem is NULL");
    if (pb->num_batches != p->nb || pb->num_reads != p->nr || pb->num_haps != p->nh)
        return fail(PH_ERR_PLAN_MISMATCH, "problem has %d batches, %d reads, %d haplotypes; plan has %d, %d, %d",
                    pb->num_batches, pb->num_reads, pb->num_haps, p->nb, p->nr, p->nh);
    if (p->P == 0) return PH_OK;
    if (!pb->batch_read_begin || !pb->batch_hap_begin || !pb->read_offset || !pb->hap_offset ||
        !pb->read_bases || !pb->hap_bases)
        return fail(PH_ERR_INVALID, "problem has a NULL array");
    return PH_OK;
}

// Adjoint configuration of a read length: 32 lanes x K <= 5 rows, then 64 x K.
bool adj_config(int m, int &P, int &K)
{
#ifdef PH_ADJ_WIDE
    if (false) {
#else
    if (m + 1 <= 32 * 5) {
#endif
        P = 32;
        K = (m + 1 + 31) / 32;
    } else if (m + 1 <= 64 * 5) {
        P = 64;
        K = std::max(3, (m + 1 + 63) / 64);
    } else {
        return false;
    }
    return adj_supported(P, K);
}

ph_status build_adjoint(ph_plan *p)
{
    if (p->adj_built) return p->adj_status;
    p->adj_built = true;
    struct Item {
        AdjRec r;
        int P, K;
    };
    std::vector<Item> items;
    items.reserve((size_t)p->P);
    std::vector<AdjRedRead> red;
    int64_t grow = 0;  // per-pair gradient rows handed out so far
    std::vector<char> has_pair(p->nr, 0);
    for (int32_t q = 0; q < p->nb; ++q) {
        const int32_t H = p->h_hb[q + 1] - p->h_hb[q];
        for (int32_t r = p->h_rb[q]; r < p->h_rb[q + 1]; ++r) {
            const int m = (int)(p->h_ro[r + 1] - p->h_ro[r]);
            int P = 0, K = 0;
            if (!adj_config(m, P, K)) {
                p->adj_status = PH_ERR_UNSUPPORTED;
                p->adj_error = "adjoint supports reads up to 319 bases";
                return p->adj_status;
            }
            if (H > 0) has_pair[r] = 1;
            // a read with several pairs: pair h's rows at grow + h m
            if (H > 1) red.push_back(AdjRedRead{grow, p->h_ro[r], m, H});
            for (int32_t h = p->h_hb[q]; h < p->h_hb[q + 1]; ++h) {
                Item it{};
                it.r.read = r;
                it.r.hap = h;
                it.r.out = (int32_t)(p->h_out_off[q] + (int64_t)(r - p->h_rb[q]) * H + (h - p->h_hb[q]));
                it.r.n = (int32_t)(p->h_ho[h + 1] - p->h_ho[h]);
                it.r.direct = H == 1 ? 1 : 0;
                it.r.grow = H == 1 ? 0 : grow + (int64_t)(h - p->h_hb[q]) * m;
                it.P = P;
                it.K = K;
                items.push_back(it);
            }
            if (H > 1) grow += (int64_t)H * m;
        }
    }
    for (int32_t r = 0; r < p->nr; ++r) p->adj_zero = p->adj_zero || !has_pair[r];
    if (red.size() >= ((size_t)1 << 31)) {
        p->adj_status = PH_ERR_UNSUPPORTED;
        p->adj_error = "too many reads with several pairs";
        return p->adj_status;
    }
    // configuration, then longest haplotype first
    std::sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
        if (a.P != b.P) return a.P > b.P;
        if (a.K != b.K) return a.K > b.K;
        if (a.r.n != b.r.n) return a.r.n > b.r.n;
        return a.r.out < b.r.out;
    });
    std::vector<AdjRec> recs(items.size());
    size_t i = 0;
    int64_t ws_total = 0;
    while (i < items.size()) {
        const int P = items[i].P, K = items[i].K, G = 64 / P;
        size_t end = i;
        while (end < items.size() && items[end].P == P && items[end].K == K) ++end;
        ph_plan::AdjRun run{P, K, (int64_t)i, (int32_t)(end - i), 0, 0, 0, 0};
        int S_max = 0;
        for (size_t a = i; a < end; a += G) {
            const size_t b = std::min(end, a + G);
            // the tile's first record has its longest haplotype
            // steps: every lane reaches column n + 2 (the absorbing row of
            // the rescaled states sums column n into column n + 2), rounded up
            // to whole checkpoint intervals
            constexpr int CK = kAdjC * kAdjR;  // steps per checkpoint
            const int S = ((items[a].r.n + P + 1 + CK - 1) / CK) * CK;
            for (size_t k = a; k < b; ++k) {
                recs[k] = items[k].r;
                recs[k].S = S;
            }
            run.ntiles += 1;
            S_max = std::max(S_max, S);
        }
        run.hs_bytes = ((S_max + P + 2 + 15) / 16) * 16;  // one code byte per column
        if ((int64_t)adj_e_bytes(P, K) + (int64_t)G * run.hs_bytes + adj_ck_lds_bytes(K) > 64 * 1024) {
            p->adj_status = PH_ERR_UNSUPPORTED;
            p->adj_error = "haplotype too long for the adjoint sweep";
            return p->adj_status;
        }
        run.ws_stride = ((int64_t)(S_max / (kAdjC * kAdjR)) * (3 * K + 3) * 64 + 63) / 64 * 64;
        const int64_t resident = (int64_t)p->cus * adj32_blocks_per_cu(P, K);
        run.grid = (int32_t)std::max<int64_t>(
            1, std::min<int64_t>({(int64_t)run.ntiles, resident, kAdjWsFloats / run.ws_stride}));
        ws_total = std::max(ws_total, (int64_t)run.grid * run.ws_stride);
        p->adj_runs.push_back(run);
        i = end;
    }
    // FP64 pass: sized for the longest haplotype and the largest class of
    // the plan; the grid is bounded by the workspace budget
    int n_max = 1, k64_max = 1;
    for (const auto &it : items) n_max = std::max(n_max, it.r.n);
    for (int32_t r = 0; r < p->nr; ++r) {
        const int m = (int)(p->h_ro[r + 1] - p->h_ro[r]);
        const int k = (m + 64) / 64;
        if (k >= 1 && k <= kAdj64Classes) {
            p->class64[k - 1] = true;
            k64_max = std::max(k64_max, k);
        }
    }
    const int S64 = ((n_max + 63 + kAdjC64 - 1) / kAdjC64) * kAdjC64;
    p->hs_bytes64 = ((S64 + 64 + 2 + 15) / 16) * 16;  // one code byte per column
    if ((int64_t)adj64_e_bytes(k64_max) + p->hs_bytes64 > 64 * 1024) {
        p->adj_status = PH_ERR_UNSUPPORTED;
        p->adj_error = "haplotype too long for the FP64 adjoint sweep";
        return p->adj_status;
    }
    p->ws64_stride = ((int64_t)(S64 / kAdjC64) * (3 * k64_max + 3) * 64 + 31) / 32 * 32;
    p->grid64 = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)p->cus * adj64_blocks_per_cu(k64_max), kAdjWs64Doubles / p->ws64_stride,
                              (int64_t)items.size()}));
    p->q64_stride = (int64_t)items.size();
    ph_status st;
    if ((st = dalloc(&p->d_adj_recs, recs.size()))) return p->adj_status = st;
    if ((st = dalloc(&p->d_ws, (size_t)std::max<int64_t>(ws_total, 1)))) return p->adj_status = st;
    if ((st = dalloc(&p->d_adj_ctr, (size_t)2 * kAdj64Classes + p->adj_runs.size()))) return p->adj_status = st;
    if ((st = dalloc(&p->d_q64, (size_t)kAdj64Classes * p->q64_stride))) return p->adj_status = st;
    if ((st = dalloc(&p->d_ws64, (size_t)p->grid64 * p->ws64_stride))) return p->adj_status = st;
    if ((st = dalloc(&p->d_grad_pair, (size_t)std::max<int64_t>(grow, 1) * 7))) return p->adj_status = st;
    if ((st = dalloc(&p->d_red, std::max<size_t>(red.size(), 1)))) return p->adj_status = st;
    p->n_red = (int32_t)red.size();
    hipError_t e = hipMemcpy(p->d_adj_recs, recs.data(), recs.size() * sizeof(AdjRec), hipMemcpyHostToDevice);
    if (e != hipSuccess) return p->adj_status = fail(PH_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
    if (!red.empty()) {
        e = hipMemcpy(p->d_red, red.data(), red.size() * sizeof(AdjRedRead), hipMemcpyHostToDevice);
        if (e != hipSuccess) return p->adj_status = fail(PH_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    return PH_OK;
}

// Longer chains make fewer, longer tiles, whose last round runs on part of
// the GPU: a plan halves the chain length (down to 1,024 columns) until it
// has this many chain tiles, 8 per wave of a launch of 3 waves per SIMD on
// 256 CUs.  (The mixed batch keeps 4,096 columns; the uniform batch, one bin
// of 64,000 reads against 8 haplotypes, gets 2,048.)
constexpr int64_t kChainMinTiles = 24576;

// The FP32 work lists of a binned plan (Section III-C), built once from the
// shape: records of every bin, bin b's range and tiles in the book image.
// A bin's records are its chain tiles, longest chain first, then single
// pairs, longest haplotype first.  A chain tile holds G = 64/P reads of one
// batch and length bin, each against the same run of the batch's
// haplotypes (at most kChainMaxHaps haplotypes and max_cols stream
// columns, every haplotype after the first at least kChainMinHap long);
// bins of fewer than 16 lanes and the reads of a batch's bin that do not
// fill a tile take single pairs.  A haplotype-length split applies to
// single pairs only (sending chains whose stream reaches the split length
// to the split's bin was slower on the mixed batch).
bool build_lists(ph_plan *p, const int32_t *rb, const int32_t *hb, const int64_t *ro, const int64_t *ho,
                 const std::vector<int64_t> &out_off, const std::vector<int16_t> &m2bin,
                 const std::vector<int16_t> &split, int max_cols, std::vector<PairRec> &recs, Book &img,
                 int64_t &chain_tile_count)
{
    const int nbins = (int)p->table.size();
    auto binP = [&](int b) { return p->table[nbins - 1 - b].P; };
    auto split_bin = [&](int b, int64_t len) {
        return (split[b] < kBuckets && hap_bucket(len) >= split[b]) ? (int)split[kMaxBins + b] : b;
    };
    // chain tiles can place the FP64 record of a pair at chain_rec_base + out
    const bool chains_ok = kChains && 2 * p->P < ((int64_t)1 << 31);
    struct Tile {
        int64_t len;   // sort key: stream or haplotype length
        int64_t first; // into `pool`
        int32_t count;
    };
    std::vector<std::vector<Tile>> chain_tiles(nbins), singles(nbins);
    std::vector<PairRec> pool;
    pool.reserve((size_t)p->P);
    std::vector<std::pair<int, int32_t>> by_bin;
    struct Seg {
        int32_t h0, H;
        int64_t len;
    };
    std::vector<Seg> segs;
    for (int32_t q = 0; q < p->nb; ++q) {
        const int32_t H = hb[q + 1] - hb[q];
        if (H == 0) continue;
        // runs of haplotypes for chains
        segs.clear();
        for (int32_t h = hb[q]; h < hb[q + 1]; ++h) {
            const int64_t n = ho[h + 1] - ho[h];
            if (!segs.empty() && n >= kChainMinHap && segs.back().H < kChainMaxHaps &&
                segs.back().len + kChainSep + n <= max_cols) {
                segs.back().H += 1;
                segs.back().len += kChainSep + n;
            } else {
                segs.push_back(Seg{h, 1, n});
            }
        }
        by_bin.clear();
        for (int32_t r = rb[q]; r < rb[q + 1]; ++r) {
            const int64_t m = ro[r + 1] - ro[r];
            by_bin.push_back({m2bin[std::min<int64_t>(m, kMaxReadLen + 1)], r});
        }
        std::stable_sort(by_bin.begin(), by_bin.end(),
                         [](const std::pair<int, int32_t> &a, const std::pair<int, int32_t> &b) { return a.first < b.first; });
        auto out_of = [&](int32_t r, int32_t h) {
            return (int32_t)(out_off[q] + (int64_t)(r - rb[q]) * H + (h - hb[q]));
        };
        auto add_single = [&](int b, int32_t r, int32_t h) {
            const int64_t n = ho[h + 1] - ho[h];
            const int bb = b == p->long_bin ? b : split_bin(b, n);
            singles[bb].push_back(Tile{n, (int64_t)pool.size(), 1});
            pool.push_back(PairRec{r, h, out_of(r, h), (int32_t)n});
        };
        size_t i = 0;
        while (i < by_bin.size()) {
            const int b = by_bin[i].first;
            size_t e = i;
            while (e < by_bin.size() && by_bin[e].first == b) ++e;
            const int cnt = (int)(e - i);
            const int G = 64 / binP(b);
            for (const Seg &sg : segs) {
                const bool chain = chains_ok && b != p->long_bin && sg.H >= 2 && binP(b) >= 16;
                const int nt = chain ? cnt / G : 0;
                for (int t = 0; t < nt; ++t) {
                    chain_tiles[b].push_back(Tile{sg.len, (int64_t)pool.size(), G});
                    for (int g = 0; g < G; ++g) {
                        const int32_t r = by_bin[i + (size_t)t * G + g].second;
                        pool.push_back(PairRec{r, sg.h0, out_of(r, sg.h0), -sg.H});
                    }
                }
                for (size_t k = i + (size_t)nt * G; k < e; ++k)
                    for (int32_t h = sg.h0; h < sg.h0 + sg.H; ++h) add_single(b, by_bin[k].second, h);
            }
            i = e;
        }
    }
    auto longest_first = [](const Tile &a, const Tile &b) { return a.len > b.len; };
    recs.clear();
    recs.reserve(pool.size());
    p->bin_tiles.assign(nbins, 0);
    p->chain_tiles = false;
    chain_tile_count = 0;
    int64_t tiles = 0;
    for (int b = 0; b < nbins; ++b) {
        std::stable_sort(chain_tiles[b].begin(), chain_tiles[b].end(), longest_first);
        std::stable_sort(singles[b].begin(), singles[b].end(), longest_first);
        img.bin_rec_begin[b] = (int32_t)recs.size();
        img.bin_tile_begin[b] = (int32_t)tiles;
        for (const Tile &t : chain_tiles[b])
            for (int g = 0; g < t.count; ++g) recs.push_back(pool[(size_t)t.first + g]);
        for (const Tile &t : singles[b]) recs.push_back(pool[(size_t)t.first]);
        const int G = 64 / binP(b);
        p->bin_tiles[b] = (int64_t)chain_tiles[b].size() + ((int64_t)singles[b].size() + G - 1) / G;
        p->chain_tiles = p->chain_tiles || !chain_tiles[b].empty();
        chain_tile_count += (int64_t)chain_tiles[b].size();
        tiles += p->bin_tiles[b];
    }
    img.bin_rec_begin[nbins] = (int32_t)recs.size();
    img.bin_tile_begin[nbins] = (int32_t)tiles;
    p->chain_rec_base = (int32_t)recs.size();
    // every pair exactly once
    std::vector<uint8_t> seen((size_t)p->P, 0);
    for (const PairRec &r : recs) {
        const int32_t cnt = r.n < 0 ? -r.n : 1;
        for (int32_t k = 0; k < cnt; ++k) {
            const int64_t o = (int64_t)r.out + k;
            if (o < 0 || o >= p->P || seen[(size_t)o]) return false;
            seen[(size_t)o] = 1;
        }
    }
    for (uint8_t v : seen)
        if (!v) return false;
    return true;
}

}  // namespace

extern "C" {

void ph_plan_opts_default(ph_plan_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rescue_threshold = 1e-28;
    o->use_graph = 1;
}

const char *ph_last_error(void) { return g_err.c_str(); }

const char *ph_version(void) { return "libpairhmm 0.1 gfx950"; }

ph_status ph_plan_create(const ph_shape *shape, const ph_plan_opts *opts_in, ph_plan **out)
{
    g_err.clear();
    if (!shape || !out) return fail(PH_ERR_INVALID, "shape or out is NULL");
    *out = nullptr;
    ph_plan_opts opts;
    if (opts_in) opts = *opts_in; else ph_plan_opts_default(&opts);
    const int32_t nb = shape->num_batches, nr = shape->num_reads, nh = shape->num_haps;
    if (nb < 0 || nr < 0 || nh < 0) return fail(PH_ERR_INVALID, "negative counts");
    if (nb > 0 && (!shape->batch_read_begin || !shape->batch_hap_begin))
        return fail(PH_ERR_INVALID, "batch arrays are NULL");
    if (!shape->read_offset || !shape->hap_offset) return fail(PH_ERR_INVALID, "offset arrays are NULL");
    if (opts.force_p && opts.force_p != 4 && opts.force_p != 8 && opts.force_p != 16 && opts.force_p != 32 &&
        opts.force_p != 64)
        return fail(PH_ERR_INVALID, "force_p must be 0, 4, 8, 16, 32 or 64");

    // --- shape validation ---------------------------------------------------
    const int32_t *rb = shape->batch_read_begin, *hb = shape->batch_hap_begin;
    const int64_t *ro = shape->read_offset, *ho = shape->hap_offset;
    if (ro[0] != 0 || ho[0] != 0) return fail(PH_ERR_INVALID, "read_offset[0] and hap_offset[0] must be 0");
    int32_t max_m = 0, max_n = 0;
    for (int32_t r = 0; r < nr; ++r) {
        int64_t m = ro[r + 1] - ro[r];
        if (m < 1) return fail(PH_ERR_INVALID, "read %d has length %lld", r, (long long)m);
        if (m > kMaxLongReadLen)
            return fail(PH_ERR_UNSUPPORTED, "read %d has length %lld > %d", r, (long long)m, kMaxLongReadLen);
        max_m = std::max<int32_t>(max_m, (int32_t)m);
    }
    for (int32_t h = 0; h < nh; ++h) {
        int64_t n = ho[h + 1] - ho[h];
        if (n < 1) return fail(PH_ERR_INVALID, "haplotype %d has length %lld", h, (long long)n);
        if (n > (1 << 30)) return fail(PH_ERR_UNSUPPORTED, "haplotype %d is too long", h);
        max_n = std::max<int32_t>(max_n, (int32_t)n);
    }
    if (nb > 0 && (rb[0] != 0 || hb[0] != 0)) return fail(PH_ERR_INVALID, "batch ranges must start at 0");
    std::vector<int64_t> out_off(nb + 1, 0);
    for (int32_t q = 0; q < nb; ++q) {
        if (rb[q + 1] < rb[q] || hb[q + 1] < hb[q] || rb[q + 1] > nr || hb[q + 1] > nh)
            return fail(PH_ERR_INVALID, "batch %d has a bad read or haplotype range", q);
        out_off[q + 1] = out_off[q] + (int64_t)(rb[q + 1] - rb[q]) * (hb[q + 1] - hb[q]);
    }
    const int64_t P = nb ? out_off[nb] : 0;
    if (P >= (int64_t)1 << 31) return fail(PH_ERR_UNSUPPORTED, "%lld pairs exceed 2^31 - 1", (long long)P);

    std::unique_ptr<ph_plan, void (*)(ph_plan *)> p(new ph_plan, free_plan);
    p->opts = opts;
    p->threshold = opts.rescue_threshold > 0 ? opts.rescue_threshold : 1e-28;
    p->nb = nb; p->nr = nr; p->nh = nh; p->P = P;
    p->nread_bases = ro[nr];
    p->nhap_bases = ho[nh];
    p->max_m = max_m;
    p->max_n = max_n;

    // --- length bins (host only: a bad table is reported before any GPU call) --
    if (opts.tune_table_path) {
        ph_status st = read_table(opts.tune_table_path, p->table);
        if (st != PH_OK) return st;
    } else if (opts.single_launch && !opts.force_p) {
        p->table = single_table();
    } else {
        p->table = default_table(opts.force_p);
    }
    if (max_m > kMaxReadLen) {
        // the longest bin: 64 lanes x 16 rows per window, never tuned
        if (opts.plain) return fail(PH_ERR_UNSUPPORTED, "plain mode supports reads up to %d bases", kMaxReadLen);
        if ((int)p->table.size() >= kMaxBins) return fail(PH_ERR_INVALID, "too many bins");
        p->table.push_back(TuneEntry{kMaxLongReadLen, 64, kLongRows / 64});
        p->long_bin = 0;  // bins are numbered longest first
        p->windows = max_m / kLongRows + 1;
    }
    const int nbins = (int)p->table.size();
    if (max_m > p->table.back().max_m)
        return fail(PH_ERR_UNSUPPORTED, "read length %d exceeds the longest configured bin (%d)", max_m,
                    p->table.back().max_m);
    std::vector<int16_t> m2bin(kMaxReadLen + 2, 0);
    for (int m = 1; m <= kMaxReadLen + 1; ++m) {
        int e = 0;
        while (e < nbins - 1 && p->table[e].max_m < m) ++e;
        m2bin[m] = (int16_t)(nbins - 1 - e);
    }
    std::vector<int32_t> binG(nbins);
    for (int b = 0; b < nbins; ++b) binG[b] = 64 / p->table[nbins - 1 - b].P;
    // haplotype-length splits: split[b] = first bucket sent to bin split[kMaxBins + b]
    // (kBuckets: none); the alt entry follows its parent, so its bin is b - 1
    std::vector<int16_t> split(2 * kMaxBins, 0);
    bool any_split = false;
    for (int b = 0; b < nbins; ++b) {
        const TuneEntry &e = p->table[nbins - 1 - b];
        split[b] = (int16_t)(e.n_split ? hap_bucket(e.n_split) : kBuckets);
        split[kMaxBins + b] = (int16_t)(e.n_split ? b - 1 : b);
        any_split = any_split || e.n_split;
    }
    int64_t cells = 0;
    for (int32_t q = 0; q < nb; ++q) {
        const int64_t H = hb[q + 1] - hb[q];
        int64_t nsum = 0;
        for (int32_t h = hb[q]; h < hb[q + 1]; ++h) nsum += ho[h + 1] - ho[h];
        for (int32_t r = rb[q]; r < rb[q + 1]; ++r) {
            const int m = (int)(ro[r + 1] - ro[r]);
            const int bin = m2bin[std::min(m, kMaxReadLen + 1)];
            cells += (int64_t)m * nsum;
            if (bin == p->long_bin) {  // every pair of the long bin gets a boundary slot
                p->long_pairs += H;
                for (int32_t h = hb[q]; h < hb[q + 1]; ++h)
                    p->bnd_stride = std::max<int64_t>(p->bnd_stride, 3 * (ho[h + 1] - ho[h] + 1));
            } else {
                p->class_pairs[rescue_class_of(m)] += H;
            }
        }
    }
    p->cells = cells;
    // the split table travels behind the length map in the same device array
    if (any_split) {
        p->split_at = (int)m2bin.size();
        m2bin.insert(m2bin.end(), split.begin(), split.end());
    }
    Book img{};
    std::vector<PairRec> recs;
    if (!opts.plain) {
        // the longest chains that still leave kChainMinTiles chain tiles (or 1,024 columns)
        for (int cols = kChainMaxCols;; cols /= 2) {
            int64_t nchain = 0;
            if (!build_lists(p.get(), rb, hb, ro, ho, out_off, m2bin, split, cols, recs, img, nchain))
                return fail(PH_ERR_INVALID, "internal: the work lists do not cover every pair once");
            if (nchain == 0 || nchain >= kChainMinTiles || cols <= 1024) break;
        }
    }
    // the first HIP calls (everything above is host work)
    HIPCHK(hipGetDevice(&p->device));
    HIPCHK(hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device));
    std::call_once(g_lut_once, [] { g_lut_status = upload_luts(); });
    HIPCHK(g_lut_status);
    p->bin_grid.assign(nbins, 0);
    for (int b = 0; b < nbins; ++b) {
        // (a chain tile can sit in a split's second bin although no single
        // pair's haplotype reaches the split: bins are launched by tiles)
        if (opts.plain || !p->bin_tiles[b] || b == p->long_bin) continue;
        const TuneEntry &e = p->table[nbins - 1 - b];
        const int64_t tiles = p->bin_tiles[b];
        const int64_t cap = (int64_t)p->cus * fwd32_blocks_per_cu(e.P, e.K);
        p->bin_grid[b] = (int)std::min<int64_t>(tiles, cap);
    }
    // side streams of the bin kernels: the long-read bin first, then the bins
    // longest reads first, round-robin, so that every stream starts with its
    // longest tiles.  (Balancing the streams' estimated work instead, largest
    // first, was 6% slower on the mixed batch.)
    {
        p->launch_order.clear();
        int next = 0;
        if (p->long_pairs) p->launch_order.push_back({p->long_bin, next++ % kSideStreams});
        for (int b = 0; b < nbins; ++b)
            if (p->bin_grid[b]) p->launch_order.push_back({b, next++ % kSideStreams});
    }
    if (p->long_pairs) {
        p->long_grid = (int)std::min<int64_t>(p->long_pairs, (int64_t)p->cus * long32_blocks_per_cu());
        p->long64_grid = (int)std::min<int64_t>(p->long_pairs, (int64_t)p->cus * long64_blocks_per_cu());
    }
    if (opts.single_launch && !opts.plain) {
        bool ok = true;
        int64_t tiles = 0;
        for (int b = 0; b < nbins; ++b) {
            if (!p->bin_tiles[b]) continue;
            const TuneEntry &e = p->table[nbins - 1 - b];
            ok = ok && single_supported(e.P, e.K);
            tiles += p->bin_tiles[b];
        }
        if (ok && tiles > 0) {
            p->single = true;
            p->single_grid = (int)std::min<int64_t>(tiles, (int64_t)p->cus * fwd32_single_blocks_per_cu());
        }
    }
    for (int c = 0; c < kRescueClasses; ++c)
        if (p->class_pairs[c])
            for (int v = 0; v < 2; ++v)
                p->rescue_grid[v][c] =
                    (int)std::min<int64_t>(p->class_pairs[c], (int64_t)p->cus * fwd64_blocks_per_cu(c, v == 0));
    p->plain_K = (max_m + 1 + 63) / 64;
    if (p->plain_K < 1) p->plain_K = 1;
    p->plain_grid = (int)std::min<int64_t>(std::max<int64_t>(P, 1), (int64_t)p->cus * plain32_blocks_per_cu(p->plain_K));

    // --- device scratch -------------------------------------------------------
    ph_status st;
    if ((st = dalloc(&p->d_out_offset, nb + 1))) return st;
    if ((st = dalloc(&p->d_m2bin, m2bin.size()))) return st;
    if ((st = dalloc(&p->d_bin_G, kMaxBins))) return st;
    if ((st = dalloc(&p->d_hist, kMaxKeys))) return st;
    // binned: the lists' records, then (chain tiles) one FP64 record slot per pair
    const int64_t nrecs = opts.plain ? P : (int64_t)recs.size() + (p->chain_tiles ? P : 0);
    if ((st = dalloc(&p->d_recs, std::max<int64_t>(nrecs, 1)))) return st;
    if ((st = dalloc(&p->d_book, 1))) return st;
    if (!opts.plain) {
        if ((st = dalloc(&p->d_book_img, 1))) return st;
        HIPCHK(hipMemcpy(p->d_book_img, &img, sizeof(Book), hipMemcpyHostToDevice));
        if (!recs.empty())
            HIPCHK(hipMemcpy(p->d_recs, recs.data(), recs.size() * sizeof(PairRec), hipMemcpyHostToDevice));
        if (p->chain_tiles && (st = dalloc(&p->d_chain_codes, (size_t)(ho[nh] + (int64_t)kChainSep * nh))))
            return st;
    }
    if ((st = dalloc(&p->d_bad, 1))) return st;
    if ((st = dalloc(&p->d_rescue, (size_t)kRescueQueues * std::max<int64_t>(P, 1)))) return st;
    if (p->long_pairs) {
        if ((st = dalloc(&p->d_bnd32, (size_t)(p->long_pairs * p->bnd_stride)))) return st;
        if ((st = dalloc(&p->d_bnd64, (size_t)(p->long_pairs * p->bnd_stride)))) return st;
        if ((st = dalloc(&p->d_long_rescue, (size_t)p->long_pairs))) return st;
    }
    HIPCHK(hipMemcpy(p->d_out_offset, out_off.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_m2bin, m2bin.data(), m2bin.size() * sizeof(int16_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_bin_G, binG.data(), nbins * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(p->d_book, 0, sizeof(Book)));

    HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    for (auto &s : p->side) HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    for (auto &e : p->join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &e : p->ev) HIPCHK(hipEventCreate(&e));
    for (auto &e : p->ev_adj) HIPCHK(hipEventCreate(&e));
    if (nb > 0) {
        p->h_rb.assign(rb, rb + nb + 1);
        p->h_hb.assign(hb, hb + nb + 1);
    }
    p->h_ro.assign(ro, ro + nr + 1);
    p->h_ho.assign(ho, ho + nh + 1);
    p->h_out_off = out_off;
    std::call_once(g_lut_adj_once, [] { g_lut_adj_status = upload_luts_adjoint(); });
    HIPCHK(g_lut_adj_status);
    if (opts.keep_checkpoints) {
        ph_status ast = build_adjoint(p.get());
        if (ast != PH_OK && ast != PH_ERR_UNSUPPORTED) return ast;
    }
    *out = p.release();
    return PH_OK;
}

ph_status ph_plan_info(const ph_plan *p, int64_t *num_pairs, int64_t *num_cells, int32_t *max_read_len,
                       int32_t *max_hap_len)
{
    if (!p) return fail(PH_ERR_INVALID, "plan is NULL");
    if (num_pairs) *num_pairs = p->P;
    if (num_cells) *num_cells = p->cells;
    if (max_read_len) *max_read_len = p->max_m;
    if (max_hap_len) *max_hap_len = p->max_n;
    return PH_OK;
}

void ph_plan_destroy(ph_plan *p) { free_plan(p); }

}  // extern "C"

namespace {

BinArgs bin_args(ph_plan *p, const ph_problem *pb)
{
    BinArgs a{};
    a.num_pairs = p->P;
    a.num_batches = p->nb;
    a.out_offset = p->d_out_offset;
    a.batch_read_begin = pb->batch_read_begin;
    a.batch_hap_begin = pb->batch_hap_begin;
    a.read_offset = pb->read_offset;
    a.hap_offset = pb->hap_offset;
    a.m2bin = p->d_m2bin;
    a.split = p->split_at >= 0 ? p->d_m2bin + p->split_at : nullptr;
    a.num_bins = (int32_t)p->table.size();
    a.bin_G = p->d_bin_G;
    a.hist = p->d_hist;
    a.recs = p->d_recs;
    a.book = p->d_book;
    return a;
}

SweepArgs sweep_args(ph_plan *p, const ph_problem *pb, const double *lin, double *out, uint8_t *status)
{
    SweepArgs a{};
    a.pb.read_offset = pb->read_offset;
    a.pb.read_bases = pb->read_bases;
    a.pb.bq = pb->base_qual;
    a.pb.iq = pb->ins_qual;
    a.pb.dq = pb->del_qual;
    a.pb.gq = pb->gcp_qual;
    a.pb.hap_offset = pb->hap_offset;
    a.pb.hap_bases = pb->hap_bases;
    a.pb.log10_params = nullptr;
    a.lin_params = lin;
    a.recs = p->d_recs;
    a.book = p->d_book;
    a.out_log10 = out;
    a.out_status = status;
    a.rescue_list = p->d_rescue;
    a.rescue_stride = std::max<int64_t>(p->P, 1);
    a.threshold = p->threshold;
    a.floor64 = std::ldexp(1.0, -1000);
    a.num_bins = (int32_t)p->table.size();
    for (int b = 0; b < a.num_bins; ++b) {
        const TuneEntry &e = p->table[a.num_bins - 1 - b];
        a.bins[b] = {e.P, e.K};
    }
    a.plain_count = (int32_t)p->P;
    a.long_bin = p->long_pairs ? p->long_bin : -1;
    a.bnd_stride = p->bnd_stride;
    a.long_rescue_list = p->d_long_rescue;
    a.chain_codes = p->d_chain_codes;
    a.chain_rec_base = p->chain_rec_base;
    a.chain_recs = p->chain_tiles ? p->d_recs + p->chain_rec_base : nullptr;
    return a;
}

// Enqueue one stage of the forward sequence on stream s:
//   0 = parameter exponentiation (explicit mode) and binning,
//   1 = FP32 sweeps of all bins, 2 = FP64 rescue sweeps.
ph_status enqueue_stage(ph_plan *p, int stage, const ph_problem *pb, const float *log10_params, double *out,
                        uint8_t *status, hipStream_t s, bool viterbi)
{
    const double *lin = log10_params ? p->d_lin : nullptr;
    SweepArgs sa = sweep_args(p, pb, lin, out, status);
    sa.viterbi = viterbi ? 1 : 0;
    if (stage == 0) {
        if (log10_params) HIPCHK(launch_prep_params(log10_params, p->nread_bases, p->d_lin, s));
        if (p->opts.plain) {
            const BinArgs ba = bin_args(p, pb);
            HIPCHK(launch_reset_keys(p->d_hist, ba.num_bins * kBuckets, p->d_book, s));
            HIPCHK(launch_plain_records(ba, s));
        } else {
            // the work lists come from plan creation: the book's bin ranges,
            // zero cursors, and the chain code stream of this call's haplotypes
            HIPCHK(launch_book_copy(p->d_book, p->d_book_img, s));
            if (p->chain_tiles)
                HIPCHK(launch_chain_codes(pb->hap_offset, pb->hap_bases, p->nh, p->d_chain_codes, s));
        }
    } else if (stage == 1) {
        if (p->opts.plain) {
            HIPCHK(launch_plain32(sa, p->plain_K, p->plain_grid, s));
        } else if (p->single && !viterbi) {
            HIPCHK(launch_fwd32_single(sa, p->single_grid, s));
        } else {
            // the bins on side streams forked from s, in the plan's launch
            // order; the windows of the long bin run in order on one stream
            HIPCHK(hipEventRecord(p->fork, s));
            bool used[kSideStreams] = {};
            for (const auto &bk : p->launch_order) {
                const int b = bk.first, k = bk.second;
                if (!used[k]) {
                    HIPCHK(hipStreamWaitEvent(p->side[k], p->fork, 0));
                    used[k] = true;
                }
                if (b == p->long_bin && p->long_pairs) {
                    SweepArgs la = sa;
                    la.bnd = p->d_bnd32;
                    for (int w = 0; w < p->windows; ++w) HIPCHK(launch_long32(la, w, p->long_grid, p->side[k]));
                } else {
                    HIPCHK(launch_fwd32(sa, sa.bins[b].P, sa.bins[b].K, b, p->bin_grid[b], p->side[k]));
                }
            }
            for (int k = 0; k < kSideStreams; ++k) {
                if (!used[k]) continue;
                HIPCHK(hipEventRecord(p->join[k], p->side[k]));
                HIPCHK(hipStreamWaitEvent(s, p->join[k], 0));
            }
        }
    } else if (!p->opts.plain) {
        for (int c = 0; c < kRescueClasses; ++c)
            if (p->rescue_grid[0][c]) HIPCHK(launch_fwd64(sa, c, true, p->rescue_grid[0][c], s));
        // after every rescaled launch: the plain queues also hold what those passed on
        for (int c = 0; c < kRescueClasses; ++c)
            if (p->rescue_grid[1][c]) HIPCHK(launch_fwd64(sa, c, false, p->rescue_grid[1][c], s));
        if (p->long_pairs) {
            SweepArgs la = sa;
            la.bnd = p->d_bnd64;
            for (int w = 0; w < p->windows; ++w) HIPCHK(launch_long64(la, w, p->long64_grid, s));
        }
    }
    return PH_OK;
}

void drop_graphs(ph_plan *p)
{
    for (int v = 0; v < 2; ++v) {
        for (int i = 0; i < 3; ++i) {
            if (p->exec[v][i]) { (void)hipGraphExecDestroy(p->exec[v][i]); p->exec[v][i] = nullptr; }
            if (p->graph[v][i]) { (void)hipGraphDestroy(p->graph[v][i]); p->graph[v][i] = nullptr; }
        }
        p->graph_key[v].clear();
    }
    if (p->adj_exec) { (void)hipGraphExecDestroy(p->adj_exec); p->adj_exec = nullptr; }
    if (p->adj_graph) { (void)hipGraphDestroy(p->adj_graph); p->adj_graph = nullptr; }
    p->adj_graph_key.clear();
}

// The adjoint's launch sequence: parameter preparation, zeroing of the
// counters (and of the gradient when some read has no pair; kernels, so that
// the sequence can be captured), one persistent FP32 launch per (P, K)
// configuration, the FP64 launches of the classes present, then the
// fixed-order sum of the per-pair rows of reads with several pairs.
ph_status enqueue_backward(ph_plan *p, const ph_problem *pb, const float *log10_params,
                           const double *grad_log10L, float *grad_params, hipStream_t s)
{
    if (log10_params) HIPCHK(launch_prep_params(log10_params, p->nread_bases, p->d_lin, s));
    if (p->adj_zero) HIPCHK(launch_zero_f32(grad_params, p->nread_bases * 7, s));
    HIPCHK(launch_zero_i32(p->d_adj_ctr, 2 * kAdj64Classes + (int)p->adj_runs.size(), s));
    AdjArgs a{};
    a.pb.read_offset = pb->read_offset;
    a.pb.read_bases = pb->read_bases;
    a.pb.bq = pb->base_qual;
    a.pb.iq = pb->ins_qual;
    a.pb.dq = pb->del_qual;
    a.pb.gq = pb->gcp_qual;
    a.pb.hap_offset = pb->hap_offset;
    a.pb.hap_bases = pb->hap_bases;
    a.lin_params = log10_params ? p->d_lin : nullptr;
    a.ws = p->d_ws;
    a.grad_in = grad_log10L;
    a.grad_out = grad_params;
    a.grad_pair = p->d_grad_pair;
    a.threshold = p->threshold;
    a.all_recs = p->d_adj_recs;
    a.q64 = p->d_q64;
    a.q64_stride = p->q64_stride;
    a.q64_count = p->d_adj_ctr;
    a.q64_next = p->d_adj_ctr + kAdj64Classes;
    a.ws64 = p->d_ws64;
    a.ws64_stride = p->ws64_stride;
    a.hs_bytes64 = p->hs_bytes64;
    a.floor64 = std::ldexp(1.0, -1000);
    for (size_t k = 0; k < p->adj_runs.size(); ++k) {
        const auto &run = p->adj_runs[k];
        a.recs = p->d_adj_recs + run.rec_begin;
        a.rec_base = run.rec_begin;
        a.nrec = run.nrec;
        a.ntiles = run.ntiles;
        a.hs_bytes = run.hs_bytes;
        a.tile_next = p->d_adj_ctr + 2 * kAdj64Classes + k;
        a.ws_stride = run.ws_stride;
        HIPCHK(launch_adj32(a, run.P, run.K, run.grid, s));
    }
    // pairs out of the FP32 range, per class (a class whose queue stayed
    // empty exits at once)
    for (int k = 1; k <= kAdj64Classes; ++k)
        if (p->class64[k - 1]) HIPCHK(launch_adj64(a, k, p->grid64, s));
    HIPCHK(launch_adj_reduce(p->d_red, p->n_red, p->d_grad_pair, grad_params, s));
    return PH_OK;
}

void drop_stage_graphs(ph_plan *p, int v)
{
    for (int i = 0; i < 3; ++i) {
        if (p->exec[v][i]) { (void)hipGraphExecDestroy(p->exec[v][i]); p->exec[v][i] = nullptr; }
        if (p->graph[v][i]) { (void)hipGraphDestroy(p->graph[v][i]); p->graph[v][i] = nullptr; }
    }
    p->graph_key[v].clear();
}

// The forward call and the Viterbi call: the same three stages, with the
// sum (forward) or the maximum (Viterbi) in the sweeps, each mode with its
// own stage graphs.
ph_status run_forward(ph_plan *p, const ph_problem *pb, const float *log10_params, double *out_log10L,
                      uint8_t *out_status, void *stream_v, bool viterbi)
{
    g_err.clear();
    if (!p) return fail(PH_ERR_INVALID, "plan is NULL");
    ph_status st = check_problem(p, pb);
    if (st != PH_OK) return st;
    if (p->P == 0) return PH_OK;
    if (!out_log10L) return fail(PH_ERR_INVALID, "out_log10L is NULL");
    if (!log10_params && (!pb->base_qual || !pb->ins_qual || !pb->del_qual || !pb->gcp_qual))
        return fail(PH_ERR_INVALID, "Phred arrays are NULL and no log10 parameters were given");
    if (viterbi && p->opts.plain) return fail(PH_ERR_UNSUPPORTED, "the Viterbi score needs a binned plan");
    hipStream_t s = (hipStream_t)stream_v;
    if (log10_params && p->lin_cap < p->nread_bases) {
        if (p->d_lin) HIPCHK(hipFree(p->d_lin));
        p->d_lin = nullptr;
        if ((st = dalloc(&p->d_lin, (size_t)p->nread_bases * 8))) return st;
        p->lin_cap = p->nread_bases;
        drop_graphs(p);
    }
    const int v = viterbi ? 1 : 0;

    // Each stage is captured into its own graph so that HIP events recorded on
    // the caller's stream between the three launches time the stages.
    if (p->opts.use_graph) {
        std::vector<const void *> key = {pb->batch_read_begin, pb->batch_hap_begin, pb->read_offset,
                                         pb->read_bases, pb->base_qual, pb->ins_qual, pb->del_qual,
                                         pb->gcp_qual, pb->hap_offset, pb->hap_bases, log10_params,
                                         out_log10L, out_status};
        if (!p->exec[v][0] || key != p->graph_key[v]) {
            drop_stage_graphs(p, v);
            for (int stage = 0; stage < 3; ++stage) {
                HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
                st = enqueue_stage(p, stage, pb, log10_params, out_log10L, out_status, p->cap, viterbi);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(p->cap, &g);
                if (st != PH_OK) { if (g) (void)hipGraphDestroy(g); drop_stage_graphs(p, v); return st; }
                if (e != hipSuccess) {
                    drop_stage_graphs(p, v);
                    return fail(PH_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
                }
                p->graph[v][stage] = g;
                e = hipGraphInstantiate(&p->exec[v][stage], g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    drop_stage_graphs(p, v);
                    return fail(PH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
                }
            }
            p->graph_key[v] = key;
        }
        for (int stage = 0; stage < 3; ++stage) {
            HIPCHK(hipEventRecord(p->ev[stage], s));
            HIPCHK(hipGraphLaunch(p->exec[v][stage], s));
        }
        HIPCHK(hipEventRecord(p->ev[3], s));
    } else {
        for (int stage = 0; stage < 3; ++stage) {
            HIPCHK(hipEventRecord(p->ev[stage], s));
            st = enqueue_stage(p, stage, pb, log10_params, out_log10L, out_status, s, viterbi);
            if (st != PH_OK) return st;
        }
        HIPCHK(hipEventRecord(p->ev[3], s));
    }
    p->last_stream = s;
    p->stages_recorded = true;
    p->forward_done = true;
    return PH_OK;
}

}  // namespace

extern "C" {

ph_status ph_forward_batch(ph_plan *p, const ph_problem *pb, const float *log10_params, double *out_log10L,
                           uint8_t *out_status, void *stream_v)
{
    return run_forward(p, pb, log10_params, out_log10L, out_status, stream_v, false);
}

ph_status ph_viterbi_batch(ph_plan *p, const ph_problem *pb, const float *log10_params, double *out_log10V,
                           uint8_t *out_status, void *stream_v)
{
    return run_forward(p, pb, log10_params, out_log10V, out_status, stream_v, true);
}

ph_status ph_backward_batch(ph_plan *p, const ph_problem *pb, const float *log10_params,
                            const double *grad_log10L, float *grad_params, void *stream_v)
{
    g_err.clear();
    if (!p) return fail(PH_ERR_INVALID, "plan is NULL");
    ph_status st = check_problem(p, pb);
    if (st != PH_OK) return st;
    if (p->P == 0) return PH_OK;
    if (!grad_log10L || !grad_params) return fail(PH_ERR_INVALID, "gradient buffers are NULL");
    if (!log10_params && (!pb->base_qual || !pb->ins_qual || !pb->del_qual || !pb->gcp_qual))
        return fail(PH_ERR_INVALID, "Phred arrays are NULL and no log10 parameters were given");
    st = build_adjoint(p);
    if (st != PH_OK) return p->adj_error.empty() ? st : fail(st, "%s", p->adj_error.c_str());
    hipStream_t s = (hipStream_t)stream_v;
    if (log10_params && p->lin_cap < p->nread_bases) {
        if (p->d_lin) HIPCHK(hipFree(p->d_lin));
        p->d_lin = nullptr;
        if ((st = dalloc(&p->d_lin, (size_t)p->nread_bases * 8))) return st;
        p->lin_cap = p->nread_bases;
        drop_graphs(p);
    }
    if (p->opts.use_graph) {
        std::vector<const void *> key = {pb->read_offset, pb->read_bases, pb->base_qual, pb->ins_qual,
                                         pb->del_qual, pb->gcp_qual, pb->hap_offset, pb->hap_bases,
                                         log10_params, grad_log10L, grad_params};
        if (!p->adj_exec || key != p->adj_graph_key) {
            if (p->adj_exec) { (void)hipGraphExecDestroy(p->adj_exec); p->adj_exec = nullptr; }
            if (p->adj_graph) { (void)hipGraphDestroy(p->adj_graph); p->adj_graph = nullptr; }
            HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
            st = enqueue_backward(p, pb, log10_params, grad_log10L, grad_params, p->cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(p->cap, &g);
            if (st != PH_OK) { if (g) (void)hipGraphDestroy(g); return st; }
            if (e != hipSuccess) return fail(PH_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            p->adj_graph = g;
            e = hipGraphInstantiate(&p->adj_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                p->adj_graph = nullptr;
                p->adj_exec = nullptr;
                return fail(PH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
            p->adj_graph_key = key;
        }
        HIPCHK(hipEventRecord(p->ev_adj[0], s));
        HIPCHK(hipGraphLaunch(p->adj_exec, s));
    } else {
        HIPCHK(hipEventRecord(p->ev_adj[0], s));
        st = enqueue_backward(p, pb, log10_params, grad_log10L, grad_params, s);
        if (st != PH_OK) return st;
    }
    HIPCHK(hipEventRecord(p->ev_adj[1], s));
    p->adj_recorded = true;
    return PH_OK;
}

ph_status ph_validate(ph_plan *p, const ph_problem *pb, void *stream_v)
{
    g_err.clear();
    if (!p) return fail(PH_ERR_INVALID, "plan is NULL");
    ph_status st = check_problem(p, pb);
    if (st != PH_OK) return st;
    hipStream_t s = (hipStream_t)stream_v;
    DevProblem d{};
    d.read_bases = pb->read_bases;
    d.hap_bases = pb->hap_bases;
    // a counter of its own: the forward's bookkeeping (rescue counts, bin
    // ranges) stays as the last forward call left it
    HIPCHK(hipMemsetAsync(p->d_bad, 0, sizeof(int32_t), s));
    HIPCHK(launch_validate(d, p->nread_bases, p->nhap_bases, p->d_bad, s));
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, p->d_bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(PH_ERR_INVALID, "%d base codes outside 0..4", bad);
    return PH_OK;
}

ph_status ph_plan_stage_ms(ph_plan *p, float ms[4])
{
    if (!p || !ms) return fail(PH_ERR_INVALID, "NULL argument");
    if (!p->stages_recorded && !p->adj_recorded) return fail(PH_ERR_STATE, "no forward or backward call recorded");
    for (int i = 0; i < 4; ++i) ms[i] = 0.0f;
    if (p->stages_recorded) {
    HIPCHK(hipEventSynchronize(p->ev[3]));
    HIPCHK(hipEventElapsedTime(&ms[0], p->ev[0], p->ev[1]));
    HIPCHK(hipEventElapsedTime(&ms[1], p->ev[1], p->ev[2]));
    HIPCHK(hipEventElapsedTime(&ms[2], p->ev[2], p->ev[3]));
    }
    if (p->adj_recorded) {
        HIPCHK(hipEventSynchronize(p->ev_adj[1]));
        HIPCHK(hipEventElapsedTime(&ms[3], p->ev_adj[0], p->ev_adj[1]));
    }
    return PH_OK;
}

ph_status ph_plan_rescued(ph_plan *p, int64_t *count)
{
    if (!p || !count) return fail(PH_ERR_INVALID, "NULL argument");
    if (!p->forward_done) return fail(PH_ERR_STATE, "no forward call recorded");
    HIPCHK(hipEventSynchronize(p->ev[3]));
    int32_t c[kRescueQueues], lc = 0, passed = 0;
    HIPCHK(hipMemcpy(c, p->d_book->rescue_count, sizeof(c), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&lc, &p->d_book->long_rescue_count, sizeof(lc), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&passed, &p->d_book->rescue_passed, sizeof(passed), hipMemcpyDeviceToHost));
    // pairs of reads longer than 1023 bases (windowed FP64 sweep), plus both
    // sets of queues, less the pairs the rescaled sweep passed on (counted twice)
    *count = lc - passed;
    for (int i = 0; i < kRescueQueues; ++i) *count += c[i];
    return PH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free forward (ph_forward_batch_noalloc): the scratch of the
// binning, the FP32 sweeps and the FP64 rescue lives in one fixed device
// array of this library instead of plan-owned buffers.  Its layout, at
// 256-byte aligned offsets: the bookkeeping (Book), the key histogram, the
// read-length -> bin map, the pairs per tile of each bin, the batch output
// offsets, the pair records, the FP64 queues and (explicit parameters) the
// linear parameters of every read base.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNaMaxPairs = (int64_t)1 << 16;
constexpr int32_t kNaMaxBatches = 1 << 14;
constexpr int64_t kNaMaxParamBases = (int64_t)1 << 16;  // explicit parameters: read bases
constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaBook = 0;
constexpr size_t kNaHist = na_align(kNaBook + sizeof(Book));
constexpr size_t kNaM2bin = na_align(kNaHist + (size_t)kMaxKeys * sizeof(int32_t));
constexpr size_t kNaBinG = na_align(kNaM2bin + (size_t)(kMaxReadLen + 2) * sizeof(int16_t));
constexpr size_t kNaOutOff = na_align(kNaBinG + (size_t)kMaxBins * sizeof(int32_t));
constexpr size_t kNaRecs = na_align(kNaOutOff + (size_t)(kNaMaxBatches + 1) * sizeof(int64_t));
constexpr size_t kNaRescue = na_align(kNaRecs + (size_t)kNaMaxPairs * sizeof(PairRec));
constexpr size_t kNaLin = na_align(kNaRescue + (size_t)kRescueQueues * kNaMaxPairs * sizeof(int32_t));
constexpr size_t kNaBytes = na_align(kNaLin + (size_t)kNaMaxParamBases * 8 * sizeof(double));

}  // namespace

// One copy per GPU, held until the process ends.  In host code this name
// is only a stand-in for the symbol: device addresses come from
// hipGetSymbolAddress (NaDevice::base).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;

// Per-device state of the allocation-free forward, set up by the first call
// on that device.
struct NaDevice {
    bool ready = false;
    unsigned char *base = nullptr;  // device address of `scratch` on this device
    int cus = 0;
    int fwd32_cap[kMaxBins] = {};   // persistent grid cap of each built-in bin (bin order)
    int fwd64_cap[2][kRescueClasses] = {};
};

std::mutex g_na_mu;
NaDevice g_na[kNaMaxDevices];
TuneEntry g_na_table[kMaxBins];  // the built-in table, shortest reads first
int g_na_bins = 0;

ph_status na_device_setup(int dev, NaDevice *&out)
{
    std::lock_guard<std::mutex> lk(g_na_mu);
    NaDevice &d = g_na[dev];
    if (!d.ready) {
        if (!g_na_bins) g_na_bins = builtin_table(g_na_table);
        // the constant tables of the sweeps (per device) and the address of
        // this device's copy of the scratch array
        HIPCHK(upload_luts());
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        HIPCHK(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
        for (int b = 0; b < g_na_bins; ++b) {
            const TuneEntry &e = g_na_table[g_na_bins - 1 - b];
            d.fwd32_cap[b] = d.cus * std::max(1, fwd32_blocks_per_cu(e.P, e.K));
        }
        for (int c = 0; c < kRescueClasses; ++c)
            for (int v = 0; v < 2; ++v) d.fwd64_cap[v][c] = d.cus * std::max(1, fwd64_blocks_per_cu(c, v == 0));
        d.base = (unsigned char *)ptr;
        d.ready = true;
    }
    out = &d;
    return PH_OK;
}

}  // namespace

extern "C" {

ph_status ph_forward_batch_noalloc(const ph_shape *shape, const ph_problem *pb, const float *log10_params,
                                   double *out_log10L, uint8_t *out_status, void *stream_v)
{
    g_err.clear();
    if (!shape || !pb) return fail(PH_ERR_INVALID, "shape or problem is NULL");
    const int32_t nb = shape->num_batches, nr = shape->num_reads, nh = shape->num_haps;
    if (nb < 0 || nr < 0 || nh < 0) return fail(PH_ERR_INVALID, "negative counts");
    if (pb->num_batches != nb || pb->num_reads != nr || pb->num_haps != nh)
        return fail(PH_ERR_PLAN_MISMATCH, "problem has %d batches, %d reads, %d haplotypes; shape has %d, %d, %d",
                    pb->num_batches, pb->num_reads, pb->num_haps, nb, nr, nh);
    if (nb > kNaMaxBatches)
        return fail(PH_ERR_UNSUPPORTED, "%d batches exceed the allocation-free maximum of %d", nb, kNaMaxBatches);
    if (nb > 0 && (!shape->batch_read_begin || !shape->batch_hap_begin))
        return fail(PH_ERR_INVALID, "batch arrays are NULL");
    if (!shape->read_offset || !shape->hap_offset) return fail(PH_ERR_INVALID, "offset arrays are NULL");
    const int32_t *rb = shape->batch_read_begin, *hb = shape->batch_hap_begin;
    const int64_t *ro = shape->read_offset, *ho = shape->hap_offset;
    if (ro[0] != 0 || ho[0] != 0) return fail(PH_ERR_INVALID, "read_offset[0] and hap_offset[0] must be 0");
    for (int32_t r = 0; r < nr; ++r) {
        const int64_t m = ro[r + 1] - ro[r];
        if (m < 1) return fail(PH_ERR_INVALID, "read %d has length %lld", r, (long long)m);
        if (m > kMaxReadLen)
            return fail(PH_ERR_UNSUPPORTED, "read %d has length %lld: the allocation-free forward takes reads up to %d",
                        r, (long long)m, kMaxReadLen);
    }
    for (int32_t h = 0; h < nh; ++h) {
        const int64_t n = ho[h + 1] - ho[h];
        if (n < 1) return fail(PH_ERR_INVALID, "haplotype %d has length %lld", h, (long long)n);
        if (n > (1 << 30)) return fail(PH_ERR_UNSUPPORTED, "haplotype %d is too long", h);
    }
    if (nb > 0 && (rb[0] != 0 || hb[0] != 0)) return fail(PH_ERR_INVALID, "batch ranges must start at 0");
    int64_t P = 0;
    for (int32_t q = 0; q < nb; ++q) {
        if (rb[q + 1] < rb[q] || hb[q + 1] < hb[q] || rb[q + 1] > nr || hb[q + 1] > nh)
            return fail(PH_ERR_INVALID, "batch %d has a bad read or haplotype range", q);
        P += (int64_t)(rb[q + 1] - rb[q]) * (hb[q + 1] - hb[q]);
    }
    if (P > kNaMaxPairs)
        return fail(PH_ERR_UNSUPPORTED, "%lld pairs exceed the allocation-free maximum of %lld", (long long)P,
                    (long long)kNaMaxPairs);
    const int64_t nbases = ro[nr];
    if (log10_params && nbases > kNaMaxParamBases)
        return fail(PH_ERR_UNSUPPORTED, "%lld read bases with explicit parameters exceed the allocation-free maximum of %lld",
                    (long long)nbases, (long long)kNaMaxParamBases);
    if (P == 0) return PH_OK;
    if (!out_log10L) return fail(PH_ERR_INVALID, "out_log10L is NULL");
    if (!pb->batch_read_begin || !pb->batch_hap_begin || !pb->read_offset || !pb->hap_offset ||
        !pb->read_bases || !pb->hap_bases)
        return fail(PH_ERR_INVALID, "problem has a NULL array");
    if (!log10_params && (!pb->base_qual || !pb->ins_qual || !pb->del_qual || !pb->gcp_qual))
        return fail(PH_ERR_INVALID, "Phred arrays are NULL and no log10 parameters were given");

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(PH_ERR_UNSUPPORTED, "device %d: too many devices", dev);
    NaDevice *d = nullptr;
    ph_status st = na_device_setup(dev, d);
    if (st != PH_OK) return st;
    const int nbins = g_na_bins;

    // pairs per bin and per FP64 class, from the host shape
    int64_t bin_pairs[kMaxBins] = {}, class_pairs[kRescueClasses] = {};
    for (int32_t q = 0; q < nb; ++q) {
        const int64_t H = hb[q + 1] - hb[q];
        for (int32_t r = rb[q]; r < rb[q + 1]; ++r) {
            const int m = (int)(ro[r + 1] - ro[r]);
            int e = 0;
            while (e < nbins - 1 && g_na_table[e].max_m < m) ++e;
            bin_pairs[nbins - 1 - e] += H;
            class_pairs[rescue_class_of(m)] += H;
        }
    }

    unsigned char *base = d->base;
    Book *book = (Book *)(base + kNaBook);
    int32_t *hist = (int32_t *)(base + kNaHist);
    int16_t *m2bin = (int16_t *)(base + kNaM2bin);
    int32_t *binG = (int32_t *)(base + kNaBinG);
    int64_t *out_off = (int64_t *)(base + kNaOutOff);
    PairRec *recs = (PairRec *)(base + kNaRecs);
    int32_t *rescue = (int32_t *)(base + kNaRescue);
    double *lin = (double *)(base + kNaLin);
    hipStream_t s = (hipStream_t)stream_v;

    BinTable tab{};
    tab.num_bins = nbins;
    for (int e = 0; e < nbins; ++e) {
        tab.max_m[e] = (int16_t)g_na_table[e].max_m;
        tab.P[e] = (int8_t)g_na_table[e].P;
    }
    // binning (the set-up kernel writes what a plan uploads at creation;
    // kernels only, so that a caller may capture the sequence)
    if (log10_params) HIPCHK(launch_prep_params(log10_params, nbases, lin, s));
    HIPCHK(launch_reset_keys(hist, nbins * kBuckets, book, s));
    HIPCHK(launch_na_setup(pb->batch_read_begin, pb->batch_hap_begin, nb, out_off, m2bin, binG, tab, s));
    BinArgs ba{};
    ba.num_pairs = P;
    ba.num_batches = nb;
    ba.out_offset = out_off;
    ba.batch_read_begin = pb->batch_read_begin;
    ba.batch_hap_begin = pb->batch_hap_begin;
    ba.read_offset = pb->read_offset;
    ba.hap_offset = pb->hap_offset;
    ba.m2bin = m2bin;
    ba.num_bins = nbins;
    ba.bin_G = binG;
    ba.hist = hist;
    ba.recs = recs;
    ba.book = book;
    HIPCHK(launch_bin_count(ba, s));
    HIPCHK(launch_bin_scan(ba, s));
    HIPCHK(launch_bin_scatter(ba, s));

    // FP32 sweeps, longest bin first, then the FP64 rescue (all on `s`)
    SweepArgs sa{};
    sa.pb.read_offset = pb->read_offset;
    sa.pb.read_bases = pb->read_bases;
    sa.pb.bq = pb->base_qual;
    sa.pb.iq = pb->ins_qual;
    sa.pb.dq = pb->del_qual;
    sa.pb.gq = pb->gcp_qual;
    sa.pb.hap_offset = pb->hap_offset;
    sa.pb.hap_bases = pb->hap_bases;
    sa.lin_params = log10_params ? lin : nullptr;
    sa.recs = recs;
    sa.book = book;
    sa.out_log10 = out_log10L;
    sa.out_status = out_status;
    sa.rescue_list = rescue;
    sa.rescue_stride = P;
    sa.threshold = 1e-28;
    sa.floor64 = std::ldexp(1.0, -1000);
    sa.num_bins = nbins;
    for (int b = 0; b < nbins; ++b) sa.bins[b] = {g_na_table[nbins - 1 - b].P, g_na_table[nbins - 1 - b].K};
    sa.plain_count = (int32_t)P;
    sa.long_bin = -1;
    for (int b = 0; b < nbins; ++b) {
        if (!bin_pairs[b]) continue;
        const int G = 64 / sa.bins[b].P;
        const int grid = (int)std::min<int64_t>((bin_pairs[b] + G - 1) / G, d->fwd32_cap[b]);
        HIPCHK(launch_fwd32(sa, sa.bins[b].P, sa.bins[b].K, b, grid, s));
    }
    for (int v = 0; v < 2; ++v)
        for (int c = 0; c < kRescueClasses; ++c)
            if (class_pairs[c])
                HIPCHK(launch_fwd64(sa, c, v == 0, (int)std::min<int64_t>(class_pairs[c], d->fwd64_cap[v][c]), s));
    return PH_OK;
}

}  // extern "C"
