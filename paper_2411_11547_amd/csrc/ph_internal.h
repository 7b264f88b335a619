// Internal declarations shared by the HIP kernels and the host runtime of
// libpairhmm.  Not part of the public ABI (that is include/ph.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ph {

// Haplotype codes: A C G T N, plus PAD for columns past the end of a
// haplotype.  PAD has emission 0 in every row, so a PAD column adds exactly
// zero to the row-m sum.
constexpr int kCodes = 6;
constexpr int kPad = 5;

// Haplotype ring buffer per lane group in LDS: 4 chunks of ring_chunk(P)
// columns plus a mirror of chunk 0, so the reads of a block of that many
// consecutive steps never wrap.  Groups of up to 32 lanes use chunks of 32
// columns: a ring of 320 bytes per group, which gives the configurations
// whose LDS sets their occupancy (16 lanes x 11-14 rows) one more wave per
// CU than chunks of 64; one 64-lane group per wave keeps chunks of 64.
constexpr int ring_chunk(int P) { return P == 64 ? 64 : 32; }
constexpr int ring_alloc(int P) { return 5 * ring_chunk(P); }

constexpr int kMaxBins = 48;             // length bins (tuned table + the long-read bin)
constexpr int kBuckets = 128;            // haplotype-length buckets per bin
constexpr int kMaxKeys = kMaxBins * kBuckets;
constexpr int kMaxReadLen = 1023;        // 64 lanes x 16 rows minus the absorbing row
constexpr int kRescueClasses = 4;        // FP64 sweep: 64 lanes x {2, 4, 8, 16} rows
// FP64 queues: [rescaled-state FP64 sweep | plain-state FP64 sweep] x class.
// The FP32 sweep queues a pair that leaves the FP32 range into the first
// set, one with a row outside the rescaled states into the second; the
// rescaled FP64 sweep passes on what leaves its own range to the second.
constexpr int kRescueQueues = 2 * kRescueClasses;
// Longer reads run in windows of kLongRows rows (64 lanes x 16 rows): the
// window's top boundary row comes from HBM, its bottom row goes back there
constexpr int kLongRows = 1024;
constexpr int kMaxWindows = 64;
constexpr int kMaxLongReadLen = kLongRows * kMaxWindows - 1;

// One read/haplotype pair: indices into the problem and into the output.
// In a chain tile of the FP32 sweep (n < 0) a record stands for the read
// against the -n haplotypes hap, hap + 1, ... of its batch, whose outputs are
// out, out + 1, ...
struct PairRec {
    int32_t read, hap, out, n;
};

// Haplotype chains.  A lane group of 16 or more lanes sweeps its read against
// several haplotypes of its batch one after the other, so that the wavefront
// fills and drains once per chain instead of once per pair.  In the chain's
// code stream every haplotype is followed by kChainSep PAD columns: the
// absorbing row has its sum two columns past the haplotype end, and lane t
// clears its states while it sweeps one of the last kChainSep - 2 of them,
// kChainSep - 2 lanes per clearing step.  The stream of haplotype h starts at
// hap_offset[h] + kChainSep h.
#ifndef PH_CHAINS
#define PH_CHAINS 1
#endif
constexpr bool kChains = PH_CHAINS;  // 0: single pairs only
constexpr int kChainSep = 6;
constexpr int kChainMaxHaps = 64;   // haplotype lengths of a chain sit one per lane
// A group clears its lanes for one boundary at a time: the boundary of every
// haplotype after a chain's first must come after the last lane of a 64-lane
// group has cleared for the previous one, so those haplotypes have at least
// 64 bases (shorter ones start a chain of their own).
constexpr int kChainMinHap = 64;
#ifndef PH_CHAIN_MAX_COLS
#define PH_CHAIN_MAX_COLS 4096
#endif
constexpr int kChainMaxCols = PH_CHAIN_MAX_COLS;  // longest chain (columns and separators)

struct DevProblem {
    const int64_t *read_offset;
    const uint8_t *read_bases, *bq, *iq, *dq, *gq;
    const int64_t *hap_offset;
    const uint8_t *hap_bases;
    const float *log10_params;  // NULL: derive from Phred
};

struct BinCfg {
    int32_t P, K;        // lanes per pair, rows per lane
};

// A bin table by value (entries shortest reads first): entry e covers reads
// up to max_m[e] bases with P[e] lanes per pair; bin b is entry
// num_bins - 1 - b (bins are numbered longest first).
struct BinTable {
    int32_t num_bins;
    int16_t max_m[kMaxBins];
    int8_t P[kMaxBins];
};

// Device-side bookkeeping written by the binning kernels and read by the
// sweeps; lives in one plan-owned buffer.
struct Book {
    int32_t bin_rec_begin[kMaxBins + 1];   // record range of every bin
    int32_t bin_tile_begin[kMaxBins + 1];  // tile range of every bin (persistent sweep)
    int32_t tile_counter;                  // plain sweep work cursor
    int32_t bin_counter[kMaxBins];         // FP32 sweep work cursor of every bin
    int32_t rescue_count[kRescueQueues];   // FP64 queue lengths
    int32_t rescue_counter[kRescueQueues]; // FP64 sweep work cursors
    int32_t rescue_passed;                 // pairs the rescaled FP64 sweep passed on
    int32_t long_counter[kMaxWindows];     // FP32 windowed passes: work cursor per window
    int32_t long64_counter[kMaxWindows];   // FP64 windowed passes: work cursor per window
    int32_t long_rescue_count;             // FP64 queue of long pairs
};

struct BinArgs {
    int64_t num_pairs;
    int32_t num_batches;
    const int64_t *out_offset;   // [num_batches+1]
    const int32_t *batch_read_begin, *batch_hap_begin;
    const int64_t *read_offset, *hap_offset;
    const int16_t *m2bin;        // [kMaxReadLen+2]
    // haplotype-length splits or NULL: split[b] = first haplotype-length
    // bucket whose pairs go to bin split[kMaxBins + b] instead of bin b
    const int16_t *split;
    int32_t num_bins;
    const int32_t *bin_G;        // pairs per tile of each bin
    int32_t *hist;               // [kMaxKeys]
    PairRec *recs;               // [num_pairs]
    Book *book;
};

struct SweepArgs {
    DevProblem pb;
    const double *lin_params;    // explicit mode: [sum m][8] linear parameters, else NULL
    const PairRec *recs;
    Book *book;
    double *out_log10;
    uint8_t *out_status;
    int32_t *rescue_list;        // [kRescueQueues][rescue_stride]
    int64_t rescue_stride;       // = num_pairs
    double threshold;            // FP32: scaled-sum rescue threshold
    double floor64;              // FP64: scaled-sum floor
    int32_t num_bins;
    BinCfg bins[kMaxBins];
    int32_t mode;                // 0 binned FP32 + rescue, 1 plain FP32, 2 FP64 rescue
    int32_t rescue_class;        // FP64: which queue
    int32_t plain_count;         // plain: number of records (tiles of 1 pair)
    // reads longer than kMaxReadLen: bin `long_bin`, windows of kLongRows rows
    int32_t long_bin;            // -1 if none
    int32_t window;              // window of this launch
    void *bnd;                   // boundary rows, [pair slot][n_max + 1][3] of T
    int64_t bnd_stride;          // elements per pair slot
    int32_t *long_rescue_list;   // FP64 queue of long pairs (record indices)
    int32_t viterbi;             // 1: max-product score (Viterbi) instead of the likelihood
    // chain tiles: the code stream, and where the FP64 records of their
    // pairs go (pair `out` of a chain at record chain_rec_base + out)
    const uint8_t *chain_codes;
    PairRec *chain_recs;
    int32_t chain_rec_base;
};

// Adjoint: one record per pair, grouped by (P, K), longest haplotype first,
// tiled G = 64/P pairs at a time; every group of a tile uses the step count S
// of the tile's first record.  A persistent workgroup takes a tile, runs its
// checkpointed forward into its own workspace slice, then the reverse sweep.
// Checkpoint layout per workgroup: [S/(CB R)][3K+3][64] values, the lane
// state (M, I, D of its K rows) and the three diagonal registers before every
// (CB R)-th step; the backward recomputes blocks of CB steps from them.
#ifndef PH_ADJ_C
#define PH_ADJ_C 4
#endif
constexpr int kAdjC = PH_ADJ_C;  // FP32: forward steps per recompute block
#ifndef PH_ADJ_R
#define PH_ADJ_R 2
#endif
constexpr int kAdjR = PH_ADJ_R;  // FP32: recompute blocks per checkpoint
constexpr int kAdjC64 = 2;  // FP64: forward steps per checkpoint block
constexpr int kAdj64Classes = 5;  // FP64 adjoint: 64 lanes x 1..5 rows

// A pair's gradient rows go to grad_out at its read's rows when the read has
// no other pair (direct = 1), else to its own rows grow .. grow + m - 1 of
// the per-pair array, which a fixed-order sum over the read's pairs reduces
// into grad_out afterwards: every row is written by exactly one pair, so the
// result does not depend on the order in which waves finish.
struct AdjRec {
    int32_t read, hap, out, n;
    int32_t S, direct;
    int64_t grow;
};

// Reads whose gradient rows sum several pairs: pair h of the read holds
// rows grow + h m .. grow + h m + m - 1 of the per-pair array.
struct AdjRedRead {
    int64_t grow;    // first per-pair row of the read's first pair
    int64_t ro;      // the read's first base (row of grad_out)
    int32_t m, H;
};

struct AdjArgs {
    DevProblem pb;
    const double *lin_params;
    const AdjRec *recs;     // records of one (P, K) configuration
    int64_t rec_base;       // index of recs[0] in all_recs
    int32_t nrec, ntiles;
    int32_t hs_bytes;       // LDS bytes per group for the staged haplotype codes (one per column)
    int32_t *tile_next;     // work cursor of this launch
    float *ws;              // [grid][ws_stride] per-workgroup checkpoints
    int64_t ws_stride;
    const double *grad_in;  // per output pair
    float *grad_out;        // per read base x 7
    float *grad_pair;       // per-pair rows x 7 (reads with several pairs)
    double threshold;       // FP32 scaled-sum range floor
    // FP64 pass over the pairs the FP32 pass left out
    const AdjRec *all_recs;
    int32_t *q64;           // [kAdj64Classes][q64_stride] indices into all_recs
    int64_t q64_stride;
    int32_t *q64_count;     // [kAdj64Classes] queue lengths
    int32_t *q64_next;      // [kAdj64Classes] work cursors
    double *ws64;           // [grid][ws64_stride] per-workgroup checkpoints
    int64_t ws64_stride;
    int32_t hs_bytes64;
    double floor64;         // FP64 scaled-sum range floor
};

hipError_t upload_luts_adjoint();
bool adj_supported(int P, int K);
int adj_e_bytes(int P, int K);
int adj_ck_lds_bytes(int K);  // FP32 pass: LDS checkpoint buffer per workgroup
hipError_t launch_adj32(const AdjArgs &a, int P, int K, int grid, hipStream_t s);
int adj32_blocks_per_cu(int P, int K);
int adj64_blocks_per_cu(int K);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
hipError_t launch_adj_reduce(const AdjRedRead *reads, int32_t nreads, const float *grad_pair, float *grad_out,
                             hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s);
int adj64_e_bytes(int K);
hipError_t launch_adj64(const AdjArgs &a, int K, int grid, hipStream_t s);

// Launchers (ph_kernels.hip).  All enqueue on `s` and return the HIP status.
hipError_t upload_luts();
hipError_t launch_bin_count(const BinArgs &a, hipStream_t s);
hipError_t launch_bin_scan(const BinArgs &a, hipStream_t s);
hipError_t launch_bin_scatter(const BinArgs &a, hipStream_t s);
hipError_t launch_plain_records(const BinArgs &a, hipStream_t s);
hipError_t launch_fwd32(const SweepArgs &a, int P, int K, int bin, int grid, hipStream_t s);
hipError_t launch_plain32(const SweepArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_fwd32_single(const SweepArgs &a, int grid, hipStream_t s);
int fwd32_single_blocks_per_cu();
bool single_supported(int P, int K);
hipError_t launch_fwd64(const SweepArgs &a, int cls, bool rescaled, int grid, hipStream_t s);
hipError_t launch_long32(const SweepArgs &a, int window, int grid, hipStream_t s);
hipError_t launch_long64(const SweepArgs &a, int window, int grid, hipStream_t s);
int long32_blocks_per_cu();
int long64_blocks_per_cu();
hipError_t launch_prep_params(const float *lg, int64_t npos, double *lin, hipStream_t s);
hipError_t launch_validate(const DevProblem &pb, int64_t nread_bases, int64_t nhap_bases,
                           int32_t *bad, hipStream_t s);
hipError_t launch_reset_keys(int32_t *hist, int nkeys, Book *book, hipStream_t s);
// chain work lists built at plan creation: the plan's book image (bin ranges,
// zero cursors) into the book, and the chain code stream of the call's haplotypes
hipError_t launch_book_copy(Book *book, const Book *image, hipStream_t s);
hipError_t launch_chain_codes(const int64_t *hap_offset, const uint8_t *hap_bases, int32_t num_haps,
                              uint8_t *codes, hipStream_t s);
hipError_t launch_na_setup(const int32_t *rb, const int32_t *hb, int32_t nb, int64_t *out_offset,
                           int16_t *m2bin, int32_t *bin_G, const BinTable &t, hipStream_t s);
int fwd32_blocks_per_cu(int P, int K);
int fwd64_blocks_per_cu(int cls, bool rescaled);
int plain32_blocks_per_cu(int K);
bool fwd32_supported(int P, int K);

}  // namespace ph
