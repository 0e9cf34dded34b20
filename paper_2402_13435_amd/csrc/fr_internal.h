// Internal declarations shared by the host runtime (fr_runtime.cpp) and the
// HIP kernels (fr_kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fr {

constexpr int kTile = 32;            // documents per matrix-core tile
constexpr int kGroup = 1024;         // documents per predicate group
constexpr int kWords = kGroup / 64;  // 64-bit mask words per group
constexpr int kNBF = 256;            // fine histogram buckets per query
constexpr int kNBC = 16;             // coarse buckets (16 fine each)
constexpr int kHist = kNBC + kNBF;   // u32 counters per query histogram
constexpr int kXcds = 8;             // work queues (one per XCD)
constexpr int kSelCap = 8192;        // candidates sorted in LDS by the select kernel
constexpr int kMaxR = 4096;          // largest K / R handled by select and rescore
// corpus groups sampled for starting thresholds: FP32 scores cost 16x the
// matrix time of BF16 ones, so the quantised forms sample more
constexpr int kTunePrewarmMs = 500;     // untimed searches before the autotuner's trials
constexpr int kSeedGroupsF32 = 32;
constexpr int kSeedGroupsLow = 64;
constexpr int kSeedGroupsMax = 128;
constexpr int kSeedBins = 2048;      // histogram buckets of the sample's scores
constexpr uint32_t kSeedTilesPerWave = 2;   // sampled tiles per query block and wavefront
// starting-threshold sample: two kept scores per 16 documents of a tile
constexpr int kSeedKeysMax = kSeedGroupsMax * (kGroup / kTile) * 4;
// Speculative starting rank: with p the share of a query's matches that lie
// in the sample, the number X of its K' best matches inside the sample is at
// most Binomial(K', p) in the tails (hypergeometric), and Bernstein's
// inequality gives P(X >= mu + t) <= exp(-t^2 / (2 (mu + t/3))), mu = K' p.
// t solves that bound for exp(-kSpecL) (kSpecL = ln 10^4): the sample's r-th
// best, r = mu + t + 1, is below the K'-th best of all matches except with
// that probability, and a failure is detected after the pass.
constexpr float kSpecL = 9.2103404f;
// Search strategies (bits; 0 = both features on), chosen by the autotuner:
// no speculative starting threshold (start from the safe one), and no
// threshold refresh by the keeper during the scan (thresholds stay at their
// start).
constexpr uint32_t kStratNoSpec = 1u;
constexpr uint32_t kStratNoRefresh = 2u;
// bits 4-7: sparse routing level L (0: off).  Queries with at most
// n_live * 2^(L-11) matches (and at most the selection size K' for the
// reduced-precision forms) skip the scan: their matching rows are listed
// from the masks and scored one by one in FP32.
constexpr uint32_t kStratSparseShift = 4u;
constexpr uint32_t kStratSparseMask = 0xF0u;
constexpr uint32_t kSparseMaxLevel = 7u;
constexpr int kLits = 12;            // literals per query in the scan's fast mask path
// device scratch of fr_search_noalloc (one array per device, in the code
// object) and the device ordinals it is looked up for
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
constexpr uint32_t kKeyNegInf = 0x007FFFFFu;  // order key of -inf
constexpr uint32_t kKeyPosInf = 0xFF800000u;  // order key of +inf

enum Dtype : int { kF32 = 0, kBF16 = 1, kFP8 = 2 };

inline int elem_bytes(int dt) { return dt == kF32 ? 4 : dt == kBF16 ? 2 : 1; }
// Bytes of one 32-row tile: rows are split into two halves of dpad/2
// elements (one per 32-lane half of a wavefront) stored as 16-byte chunks in
// [chunk][lane][16 B] order, so a wavefront loads a chunk as one contiguous
// kilobyte.
inline size_t tile_bytes(int dt, int dpad) { return (size_t)kTile * dpad * elem_bytes(dt); }

// ---------------------------------------------------------------- kernels
struct TileRowsArgs {
  const float* rows;       // n x dim FP32 row-major (device)
  uint64_t n;
  uint32_t dim, dpad, dt;
  const uint32_t* slots;   // destination slot of each row, or null -> slot_base + i
  uint64_t slot_base;
  uint8_t* tiles;          // tiled storage of the destination
  float* scale;            // FP8: per-row scale out (indexed by slot); may be null otherwise
  float* master;           // optional FP32 row copy [slot][dpad]
  float* norm;             // optional per-row L2 norm out (indexed by i)
  uint32_t* norm_max;      // optional running max of norms (float bits)
  const uint32_t* n_dev;   // optional device row count (min with n)
};

struct TermArgs {
  const uint64_t* off;     // n + 1 offsets into terms
  const uint32_t* terms;
  const uint32_t* slots;   // slot of each row, or null -> slot_base + i
  uint64_t slot_base;
  uint64_t n;
  uint64_t* bits;          // [groups][vocab][16]
  uint32_t vocab;
  int set;                 // 1: set bits, 0: clear bits
};

struct LiveArgs {
  const uint32_t* slots;   // or null -> slot_base + i
  uint64_t slot_base;
  uint64_t n;
  const uint32_t* ids;     // id per row (set) or null (clear)
  uint32_t* slot_ids;
  uint64_t* live;
  int set;
};

struct PrepArgs {
  uint32_t max_q;          // grid size (queries the workspace can hold)
  const uint32_t* n_dev;   // device: queries in this batch
  const uint32_t* k;       // requested K per query
  uint32_t* kp;            // first-pass selection size per query (out)
  uint32_t dt;
  uint32_t rescore_r, rescore_min;
  const float* qnorm;      // per-query norm
  const uint32_t* norm_max;
  uint32_t* tau;
  uint32_t* tsafe;         // safe starting key when the start is speculative, else 0
  uint32_t* cnt;
  uint32_t* smax;
  uint32_t* hist;
  float* hlo;
  float* hinvw;
  unsigned long long* nmatch;
  uint32_t* qlist;
  uint32_t* n_list;        // device: first-pass list length (= n_q)
  uint32_t* n_list2;       // device: rerun list length (zeroed)
  uint32_t* work;          // kXcds counters (zeroed)
  uint32_t* ovf;           // per-query overflow flag
  // CNF of the batch and its per-query literal table (out): kLits term ids
  // per query, and an info word: bits 0-4 literal count (<= kLits), 8-23
  // first-literal-of-clause flags, 24 an empty clause, 25 more than kLits
  // literals (evaluated from the CSR arrays instead), 26 at least one clause.
  const uint32_t* clause_off;
  const uint32_t* literal_off;
  const uint32_t* terms;
  uint32_t* lit;
  uint32_t* linfo;
};


// Predicate masks of one search pass, precomputed for the scan: word w of
// group g for the query at position p of the pass's list is
// mw[(g * kWords + w) * ppad + p].  Optionally adds each query's matches to
// nmatch.
struct MaskWordArgs {
  const uint32_t* qlist;
  const uint32_t* n_list;  // device: positions in the list
  uint32_t max_list;       // grid size (positions)
  uint32_t ppad;           // row stride of mw (>= positions, multiple of 256)
  uint32_t n_groups;
  uint32_t gpt;            // groups per thread
  const uint64_t* live;
  const uint64_t* bits;
  uint32_t vocab;
  const uint32_t* lit;     // per-query literal table (see PrepArgs)
  const uint32_t* linfo;
  const uint32_t* clause_off;
  const uint32_t* literal_off;
  const uint32_t* terms;
  uint64_t* mw;
  unsigned long long* nmatch;
  uint32_t count_matches;
  const uint32_t* run_if;  // device flag, or null: when *run_if == 0 the pass does nothing
};

// Starting thresholds: for each query of the first pass, the K'-th best
// score among the matches in the first few groups (less a rounding margin)
// is a lower bound of its final K'-th best score (the safe start); the r-th
// best for a smaller r (see kSpecL) is a tighter, speculative start.
struct SeedArgs {
  const uint32_t* qlist;
  const uint32_t* n_list;  // device
  uint32_t max_list;       // grid size (positions)
  const uint32_t* kp;
  const uint8_t* tiles;
  const float* xscale;     // FP8 row scales or null
  const uint8_t* qtiles;
  const float* qscale;     // FP8 query scales or null
  const float* qnorm;
  const uint32_t* norm_max;
  const uint64_t* mw;      // the pass's masks (see MaskWordArgs)
  uint32_t ppad;
  uint32_t n_groups;       // groups sampled (the first n_groups of the corpus)
  uint32_t dim;
  uint32_t* skey;          // [list position][row] kept sample score keys (0: none)
  uint32_t row;            // skey row stride, >= n_groups * 128
  const unsigned long long* nmatch;   // matches of each query (whole corpus)
  uint32_t* tau;
  uint32_t* tsafe;         // safe start when tau's start is speculative, else 0
  float* hlo;              // histogram range of the scan (narrowed here)
  float* hinvw;
  uint32_t strategy;       // kStrat* bits
};

struct ScanArgs {
  const uint8_t* tiles;
  const float* xscale;     // FP8 row scales or null
  const uint64_t* live;
  const uint64_t* bits;
  uint32_t vocab;
  uint32_t n_groups;
  const uint8_t* qtiles;
  const float* qscale;     // FP8 query scales or null
  const uint32_t* qlist;
  const uint32_t* n_list;  // device
  const uint32_t* kp;
  uint32_t* tau;
  uint32_t* cnt;
  uint32_t* smax;
  uint32_t* hist;
  const float* hlo;
  const float* hinvw;
  unsigned long long* cand_key;  // [q][cap]: score key << 32 | slot
  uint32_t cap;
  uint32_t* work;
  uint32_t tpi;            // tiles per work item (a multiple of 4)
  const uint64_t* mw;      // predicate masks of the pass (see MaskWordArgs)
  uint32_t ppad;
  uint32_t strategy;       // kStrat* bits
};

// Exact selection of a pass's candidates.  The first pass also sets up the
// second one for the queries it cannot answer: those whose candidate buffer
// overflowed keep their (safe, tightened) threshold with the histogram range
// narrowed to [tau, max seen]; those whose speculative starting threshold
// proved too high restart from the safe one.  Their counters are cleared and
// they are appended to qlist2.
struct SelectArgs {
  const uint32_t* qlist;
  const uint32_t* n_list;  // device
  uint32_t max_list;       // grid size
  int final_pass;          // overflow here is final: mark the query failed
  const uint32_t* kp;
  uint32_t* tau;
  uint32_t* cnt;
  uint32_t* smax;
  uint32_t* hist;
  float* hlo;
  float* hinvw;
  uint32_t* qlist2;        // second pass list (first pass appends)
  uint32_t* n_list2;
  uint32_t* work;          // work counters, zeroed for the second scan
  const float* qnorm;
  const uint32_t* norm_max;
  const unsigned long long* cand_key;   // score key << 32 | slot
  const uint32_t* slot_ids;            // slot -> external id
  uint32_t cap;
  unsigned long long* sel_key;   // [q][rmax]: score key << 32 | ~id
  uint32_t* sel_slot;
  uint32_t* sel_cnt;
  uint32_t rmax;
  uint32_t* ovf;           // final pass: 1 where the query failed
  uint32_t* tsafe;         // first pass: nonzero where the start was speculative
  // direct output (FP32 path)
  int write_out;
  const uint32_t* k;
  uint32_t k_max;
  uint32_t* out_ids;
  float* out_scores;
  uint32_t* out_count;
  const unsigned long long* nmatch;
  unsigned long long* out_nmatch;
};

struct RescoreArgs {
  uint32_t max_q;
  const uint32_t* n_dev;
  const uint32_t* ovf;
  const float* master;     // [slot][dpad]
  const float* qrows;      // [q][dpad]
  uint32_t dpad;
  const unsigned long long* sel_key;
  const uint32_t* sel_slot;
  const uint32_t* sel_cnt;
  uint32_t rmax;
  const uint32_t* k;
  uint32_t k_max;
  uint32_t* out_ids;
  float* out_scores;
  uint32_t* out_count;
  const unsigned long long* nmatch;
  unsigned long long* out_nmatch;
};


// ---- sign-code pre-selection (fr_quant.hip) ----------------------------
// Codes of n_bits (64, 128, 256 or 512) per row.  The corpus layout keeps
// the words of 64 consecutive slots together: word w of slot s is at
// codes[((s / 64) * W + w) * 64 + s % 64], W = n_bits / 64, so a wavefront
// reads one word of 64 documents as 512 contiguous bytes.
constexpr int kQuantQB = 32;        // queries per block of the code scans
constexpr uint32_t kQuantAll = 1u;  // take every tie at the threshold
constexpr uint32_t kQuantFail = 2u; // more ties at the threshold than the tie buffer
constexpr uint32_t kQuantMaxK = 1u << 16;  // most survivors per query

struct SignArgs {
  const float* rows;       // FP32 rows, `ld` floats apart
  uint32_t ld;
  uint64_t n;              // rows
  const uint32_t* n_dev;   // device row count (min with n), or null
  const uint32_t* slots;   // corpus slot of each row, or null -> slot_base + i
  uint64_t slot_base;
  const uint32_t* bin_off; // [n_bits + 1]: bit j sums entries bin_off[j] .. bin_off[j+1]
  const uint32_t* bin_dim; //   of (coordinate, sign)
  const float* bin_sign;
  uint32_t dim;            // coordinates a row holds (bin_dim < dim)
  uint32_t n_bits;
  uint64_t* codes;
  int corpus_layout;       // 1: corpus layout (above); 0: [row][W]
};

struct QuantArgs {
  const uint64_t* codes;   // corpus codes
  const uint64_t* qcode;   // [q][W]
  const uint64_t* mw;      // predicate masks [(group * 16 + word) * ppad + q]
  uint32_t ppad;
  uint32_t n_slices;       // 64-document slices scanned (16 per group)
  uint32_t spb;            // slices per thread block
  uint32_t max_q;          // grid size (queries)
  const uint32_t* n_dev;   // device: queries in the batch
  uint32_t n_bits;
  uint32_t* hist;          // [q][n_bits + 1] matches per score (histogram pass)
  const uint32_t* thr;     // collect pass: per-query threshold score
  const uint32_t* flag;    //   kQuantAll / kQuantFail
  uint32_t* cnt;           //   survivors per query
  uint32_t* surv;          //   [q][scap] survivor slots
  uint32_t scap;
  uint32_t* ntie;          //   ties at the threshold per query
  uint32_t* ties;          //   [q][tcap]
  uint32_t tcap;
};

struct QuantSelectArgs {
  uint32_t max_q;
  const uint32_t* n_dev;
  const uint32_t* k;
  uint32_t factor;         // quantK = factor * k, at most scap
  uint32_t n_bits;
  const uint32_t* hist;
  uint32_t* thr;
  uint32_t* need;          // ties to take at the threshold
  uint32_t* flag;
  uint32_t* cnt;
  uint32_t* ntie;
  const uint32_t* ties;
  uint32_t* surv;
  uint32_t scap, tcap;
  const uint32_t* slot_ids;
  // state of the exact selection that follows (no bucket cut, no rerun)
  uint32_t* tau;
  float* hinvw;
  uint32_t* tsafe;
  uint32_t* ovf;
};

// FP32 inner products of listed rows (the pre-selection's survivors, or a
// sparse-routed query's matches) against the query: row i of query q is
// slot rows[q * stride + i], i < cnt[q]; cnt[q] > stride marks a failed query
// (skipped).  Queries are y < max_q, or qlist[y] for y < *n_list when a
// list is given.
struct RowDotArgs {
  uint32_t max_q;
  const uint32_t* n_dev;
  const uint32_t* qlist;   // or null
  const uint32_t* n_list;
  const uint32_t* cnt;
  const uint32_t* rows;
  uint32_t stride;
  uint32_t max_cnt;        // grid size: most rows of any query
  const float* master;     // [slot][dpad], or null: FP32 embedding tiles
  const uint8_t* tiles;
  uint32_t dpad;
  const float* qrows;      // [q][q_ld]
  uint32_t q_ld;
  uint32_t dim;
  unsigned long long* key; // [q][key_stride]: FP32 score key << 32 | slot
  uint32_t key_stride;     // >= stride
  // optional (null: none): each score into the query's selection histogram
  // over [hlo, hlo + kNBF / hinvw], as the scan bins its candidates, so that
  // the exact selection can cut before sorting
  uint32_t* hist;
  const float* hlo;
  const float* hinvw;
};

// Sparse routing: split the batch (queries 0..n-1, whose masks were just
// computed at position = query) into the scan's list and the sparse list,
// keeping query order in both.
struct RouteArgs {
  uint32_t max_q;
  const uint32_t* n_dev;
  const unsigned long long* nmatch;
  const uint32_t* kp;      // with cap_by_kp: a query routes only if n_match <= kp
  int cap_by_kp;
  uint32_t limit;          // route queries with n_match <= limit
  uint32_t* qlist;         // out: the scan's queries
  uint32_t* n_list;
  uint32_t* slist;         // out: the sparse queries
  uint32_t* n_slist;
};

// The matching slots of each sparse query, from its mask words (stored at
// position = query), appended to rows[q * cap ...] with cnt[q] counting.
struct SparseRowsArgs {
  uint32_t max_q;
  const uint32_t* slist;
  const uint32_t* n_slist;
  const uint64_t* mw;
  uint32_t ppad;
  uint32_t n_groups;
  uint32_t gpb;            // groups per block
  uint32_t* cnt;
  uint32_t* rows;
  uint32_t cap;
};

// Codes of a.n rows.
hipError_t launch_sign_codes(const SignArgs& a, hipStream_t s);
// Histogram pass: per query, matches per code-agreement score.
hipError_t launch_quant_hist(const QuantArgs& a, hipStream_t s);
// Per query: the threshold score that keeps quantK survivors, and the ties
// to take at it; resets the survivor and tie counters.
hipError_t launch_quant_cut(const QuantSelectArgs& a, hipStream_t s);
// Collect pass: survivors above the threshold (and every tie when all are
// taken), ties at the threshold to their own buffer.
hipError_t launch_quant_collect(const QuantArgs& a, hipStream_t s);
// The `need` lowest-id ties join the survivors; a failed query gets a count
// above scap (the exact selection then marks it failed).
hipError_t launch_quant_ties(const QuantSelectArgs& a, hipStream_t s);
// FP32 inner products of listed rows (fr_sparse.hip).
hipError_t launch_row_dots(const RowDotArgs& a, hipStream_t s);
hipError_t launch_route(const RouteArgs& a, hipStream_t s);
hipError_t launch_sparse_rows(const SparseRowsArgs& a, hipStream_t s);

// ---- term lists for large vocabularies (fr_lists.hip) ------------------
// An index created with list_terms = L keeps each document's terms as a
// list of at most L ids, laid out [slot/64][j][slot%64] (term j of 64
// consecutive slots contiguous), with a count per slot, instead of one
// bitmap per vocabulary term.  A search first materialises bitmaps for the
// batch's own distinct terms only (the dictionary, sorted; literals are
// renumbered to dictionary indices on the host), in the layout of the
// per-term bitmaps: [group][n_dict][16 words].
constexpr uint32_t kBatchTermsMax = 1024;

struct ListWriteArgs {
  const uint64_t* off;     // n + 1 offsets into terms
  const uint32_t* terms;
  const uint32_t* slots;   // slot of each row, or null -> slot_base + i
  uint64_t slot_base;
  uint64_t n;
  uint32_t* tlist;
  uint32_t* tcnt;
  uint32_t L;
};

struct BatchBitsArgs {
  const uint32_t* tlist;
  const uint32_t* tcnt;
  uint32_t L;
  uint32_t n_groups;
  const uint32_t* dict;    // sorted distinct terms of the batch
  uint32_t n_dict;         // <= kBatchTermsMax
  uint64_t* bits;          // out: [group][n_dict][16]
};

hipError_t launch_list_write(const ListWriteArgs& a, hipStream_t s);
hipError_t launch_batch_bits(const BatchBitsArgs& a, hipStream_t s);

// Launchers (fr_kernels.hip).  Each returns the HIP error of the launch.
hipError_t launch_tile_rows(const TileRowsArgs& a, hipStream_t s);
hipError_t launch_terms(const TermArgs& a, hipStream_t s);
hipError_t launch_live(const LiveArgs& a, hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
// Query tiling (t, over the batch's rows) fused with the per-query state of
// launch_prep (a); t.n == a.max_q and t.n_dev == a.n_dev.
hipError_t launch_query_prep(const TileRowsArgs& t, const PrepArgs& a, hipStream_t s);
hipError_t launch_mask_words(const MaskWordArgs& a, hipStream_t s);
hipError_t launch_seed(const SeedArgs& a, int dt, int dpad, hipStream_t s);
hipError_t launch_zero_work(uint32_t* work, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, int dt, int dpad, int qb, int nw, int n_wg,
                       hipStream_t s);
hipError_t launch_select(const SelectArgs& a, hipStream_t s);
hipError_t launch_rescore(const RescoreArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
// flag |= 1 if any of x[0..n) is not finite.
hipError_t launch_check_finite(const float* x, uint64_t n, uint32_t* flag, hipStream_t s);
// Device address of the no-allocation scratch (kScratchBytes) on `device`,
// which must be the current device; looked up once per device.
hipError_t scratch_address(int device, void** out);
// Scan variants: query blocks of 32 per wavefront x wavefronts per workgroup.
bool scan_supported(int dt, int dpad, int qb, int nw);

}  // namespace fr
