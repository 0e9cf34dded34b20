// Host runtime of the filtered top-K retrieval library: the C ABI of
// include/fr.h, input validation, the slot store (id map, free slots,
// epochs), pre-allocated workspaces, and the launch sequence of a search.
//
// Every device allocation happens in fr_create (appendix "Memory
// Pre-Allocation"); later calls only validate, copy and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "fr.h"
#include "fr_host.h"
#include "fr_internal.h"

using namespace fr;

namespace {

thread_local std::string g_err;

fr_status fail(fr_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define FR_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ix->failed = true;                                                              \
      return fail(FR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    }                                                                                 \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count, std::vector<void*>& owned) {
  void* v = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  hipError_t e = hipMalloc(&v, bytes);
  if (e == hipSuccess) owned.push_back(v);
  *p = (T*)v;
  return e;
}

template <class T>
hipError_t halloc(T** p, size_t count, std::vector<void*>& owned) {
  void* v = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  hipError_t e = hipHostMalloc(&v, bytes, hipHostMallocDefault);
  if (e == hipSuccess) owned.push_back(v);
  *p = (T*)v;
  return e;
}

uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

}  // namespace

struct Workspace {
  // sizes the buffers below were laid out for: queries, clauses and
  // literals per search, row stride of the masks, candidate slots per query
  uint32_t qcap = 0, cmax = 0, lmax = 0, ppad = 0, cand_cap = 0;
  // device
  float* qrow = nullptr;
  uint8_t* qtiles = nullptr;
  float* qscale = nullptr;
  float* qnorm = nullptr;
  // per-search inputs, one block copied from its pinned twin at once:
  // [desc 4][k qmax][clause_off qmax+1][literal_off cmax+1][terms lmax]
  uint32_t* in = nullptr;
  uint32_t* clause_off = nullptr;
  uint32_t* literal_off = nullptr;
  uint32_t* terms = nullptr;
  uint32_t* k = nullptr;
  uint32_t* kp = nullptr;
  uint32_t* tau = nullptr;
  uint32_t* cnt = nullptr;
  uint32_t* smax = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* qlist = nullptr;
  uint32_t* qlist2 = nullptr;
  uint32_t* ovf = nullptr;
  uint32_t* sel_cnt = nullptr;
  uint32_t* lit = nullptr;
  uint32_t* linfo = nullptr;
  uint32_t* desc = nullptr;  // [0] n_q, [1] n_list, [2] n_list2
  uint32_t* work = nullptr;
  float* hlo = nullptr;
  float* hinvw = nullptr;
  unsigned long long* nmatch = nullptr;
  unsigned long long* cand_key = nullptr;
  uint64_t* mw = nullptr;    // predicate masks of the current pass
  uint32_t* skey = nullptr;   // kept sample scores of the starting thresholds
  uint32_t* tsafe = nullptr;  // safe starting thresholds behind speculative ones
  unsigned long long* sel_key = nullptr;
  uint32_t* sel_slot = nullptr;
  uint32_t* out_ids = nullptr;
  float* out_scores = nullptr;
  uint32_t* out_count = nullptr;
  unsigned long long* out_nmatch = nullptr;
  // pinned host staging (h_in mirrors in)
  uint32_t* h_in = nullptr;
  float* h_q = nullptr;
  uint32_t* h_co = nullptr;
  uint32_t* h_lo = nullptr;
  uint32_t* h_terms = nullptr;
  uint32_t* h_k = nullptr;
  uint32_t* h_desc = nullptr;
  uint32_t* h_ids = nullptr;
  float* h_scores = nullptr;
  uint32_t* h_count = nullptr;
  unsigned long long* h_nmatch = nullptr;
  uint32_t* h_cnt = nullptr;
  uint32_t* h_selcnt = nullptr;
  uint32_t* h_desc_out = nullptr;  // device descriptor after the call ([2] = rerun list)
  // sign-code pre-selection (indexes with sign codes)
  uint64_t* qcode = nullptr;   // [q][W] query codes
  uint32_t* qhist = nullptr;   // [q][bits + 1] matches per code score
  uint32_t* qthr = nullptr;
  uint32_t* qneed = nullptr;
  uint32_t* qflag = nullptr;
  uint32_t* ntie = nullptr;
  uint32_t* surv = nullptr;    // [q][scap]
  uint32_t* ties = nullptr;    // [q][tcap]
  unsigned long long* qkey = nullptr;   // [q][scap]
  // term lists: the batch dictionary (device + pinned twin, after the input
  // block) and the bitmaps of its terms
  uint32_t* dict = nullptr;
  uint32_t* h_dict = nullptr;
  uint64_t* bbits = nullptr;
  uint32_t n_dict = 0;
  // sparse routing: the sparse queries and their matching rows
  uint32_t* slist = nullptr;
  uint32_t* srows = nullptr;   // [q][rcap]
  bool last_preselect = false;
  uint64_t last_survivors = 0;
  hipEvent_t done = nullptr, e_scan0 = nullptr, e_scan1 = nullptr, e_end = nullptr;
  // the event that marks the end of the workspace's last call: its timing
  // ring's end event for a search (one event record for both purposes),
  // else `done`
  hipEvent_t fin = nullptr;
  hipEvent_t e_start = nullptr;   // recorded before the call's input upload
  // timing ring: scan start / scan end / end of the search, per recent call
  static constexpr int kRing = 64;
  hipEvent_t r0[kRing] = {}, r1[kRing] = {}, r2[kRing] = {}, r3[kRing] = {};
  uint64_t n_calls = 0;
  // captured search sequence (FR_GRAPH), valid for one tiling / corpus
  // extent / output binding
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t gkey[10] = {};
  bool in_flight = false;
  uint32_t last_nq = 0;
  double last_alg_bytes = 0, last_alg_flops = 0;
  uint64_t last_terms = 0, last_live = 0;
};

struct fr_index {
  fr_config cfg{};
  int dt = 0;
  uint32_t dim = 0, dpad = 0;
  uint64_t cap = 0;        // slots, multiple of kGroup
  uint32_t rmax = 0;       // per-query selection buffer (max of k_max and R)
  uint32_t r = 0, r_min = 0;
  uint32_t cand_cap = 0;
  // sign codes: bits per document (0: none), quantK = factor * k (at most
  // scap), tie buffer per query, the corpus codes and the encoding table
  uint32_t qbits = 0, qfactor = 0, scap = 0, tcap = 0;
  // term lists (list_terms > 0) instead of per-term bitmaps
  uint32_t L = 0, batch_terms = 0;
  uint32_t* tlist = nullptr;
  uint32_t* tcnt = nullptr;
  uint64_t* codes = nullptr;
  uint32_t* d_bin_off = nullptr;
  uint32_t* d_bin_dim = nullptr;
  float* d_bin_sign = nullptr;
  uint64_t bin_cap = 0;     // table entries reserved
  bool quant_set = false;   // fr_set_quantizer was called
  uint32_t qmax = 0, cmax = 0, lmax = 0;
  uint32_t seed_groups = 0;   // corpus groups sampled for starting thresholds
  int n_cu = 0, n_wg = 0;
  int qb = 0, nw = 0, gpi = 0;   // 0: chosen per batch
  uint32_t strat = 0;             // search strategy bits (FR_STRAT_*)
  bool strat_pinned = false;      // fr_set_strategy was called
  // autotuned choices keyed by (Q bucket, K' bucket, selectivity bucket);
  // the index's arch, dtype, dimension and vocabulary complete the key
  struct Tuned {
    int qb, nw, gpi;
    uint32_t strat;
    float ms;
  };
  std::map<std::tuple<int, int, int>, Tuned> tuned;
  int last_sel = -1;              // selectivity bucket of the last host-output search
  char arch[32] = {};
  hipStream_t stream = nullptr;
  std::vector<void*> dev_owned, host_owned;
  // corpus
  uint8_t* tiles = nullptr;
  float* xscale = nullptr;
  float* master = nullptr;
  uint32_t* slot_ids = nullptr;
  uint64_t* live = nullptr;
  uint64_t* bits = nullptr;
  uint32_t* norm_max = nullptr;
  uint32_t* d_flag = nullptr;
  // load / update staging
  uint64_t stage_rows = 0, stage_terms = 0;
  float* d_rows = nullptr;
  uint64_t* d_off = nullptr;
  uint32_t* d_tl = nullptr;
  uint32_t* d_ids = nullptr;
  uint32_t* d_slots = nullptr;
  uint32_t* h_flag = nullptr;
  // update staging: device buffers and their pinned host twins for one
  // chunk of an update (inserted rows, ids, term CSR, slots; deleted slots
  // and their term CSR), so that an update is enqueued without waiting
  uint64_t ustage_rows = 0, ustage_terms = 0;
  float* d_urows = nullptr;
  uint64_t* d_uoff = nullptr;
  uint32_t *d_uterms = nullptr, *d_uids = nullptr, *d_uslots = nullptr;
  uint32_t *d_dslots = nullptr, *d_dterms = nullptr;
  uint64_t* d_doff = nullptr;
  float* h_urows = nullptr;
  uint64_t* h_uoff = nullptr;
  uint32_t *h_uterms = nullptr, *h_uids = nullptr, *h_uslots = nullptr;
  uint32_t *h_dslots = nullptr, *h_dterms = nullptr;
  uint64_t* h_doff = nullptr;
  hipEvent_t ustage_free = nullptr;   // the staging's last copies are done
  hipEvent_t upd_done = nullptr;      // the last update's device work is done
  bool ustage_pending = false, upd_pending = false;
  // host copy of every slot's term list (so a delete clears exactly the
  // document's term bits): slot s holds t_arena[t_off[s] .. + t_len[s])
  std::vector<uint32_t> t_arena;
  std::vector<uint64_t> t_off;
  std::vector<uint32_t> t_len;
  uint64_t t_garbage = 0;
  // host mirror of the slot store
  std::unordered_map<uint32_t, uint32_t> id2slot;
  std::vector<uint32_t> slot_id;
  std::priority_queue<uint32_t, std::vector<uint32_t>, std::greater<uint32_t>> free_slots;
  uint64_t hwm = 0, n_live = 0, epoch = 0;
  std::vector<Workspace> ws;
  size_t next_ws = 0;
  bool failed = false;
  fr_search_stats last{};
  bool have_last = false;
  size_t last_ws = 0;
  std::vector<std::pair<uint32_t, uint32_t>> history;  // (workspace, ring slot) per call
  // fr_search_noalloc: the device's scratch array, a pinned input block
  // (sized like a workspace's) with the event of its last copy, and a pinned
  // count buffer for the synchronous failure check
  uint8_t* scratch = nullptr;
  uint32_t* na_h_in = nullptr;
  uint32_t* na_h_count = nullptr;
  hipEvent_t na_copied = nullptr;
  hipEvent_t na_done = nullptr;   // end of the last scratch-array search
  bool na_pending = false, na_inflight = false;
  std::mutex mu;
};

namespace {

// row stride (keys) of a workspace's starting-threshold sample: four kept
// scores per sampled tile
uint32_t seed_row(const fr_index* ix) { return ix->seed_groups * (kGroup / kTile) * 4u; }

template <class T>
void carve(T** p, uint8_t* base, size_t& off, size_t count) {
  *p = base ? (T*)(base + off) : nullptr;
  off += (std::max<size_t>(count * sizeof(T), 1) + 255) / 256 * 256;
}

// Device buffers of a search workspace for qm queries, cm clauses and lm
// literals per search over n_groups corpus groups, laid out in one block at
// `base` (256-byte aligned pieces); `outputs` adds the result buffers that
// host-pointer searches copy back from.  Sets the workspace's sizes and
// returns the block's size; with base == nullptr it only computes it.
bool strategy_ok(uint32_t st) {
  return !(st & ~(uint32_t)(FR_STRAT_NO_SPECULATION | FR_STRAT_NO_REFRESH | FR_STRAT_SPARSE_MASK)) &&
         ((st & FR_STRAT_SPARSE_MASK) >> 4) <= kSparseMaxLevel;
}

// Most rows a sparse-routed query can have: the candidate buffer (FP32), or
// the selection size R (the reduced-precision forms route a query only when
// all its matches fit in R, so their result is the one the scan would give).
uint32_t sparse_cap(const fr_index* ix) { return ix->dt == kF32 ? ix->cand_cap : ix->rmax; }

size_t layout_workspace(const fr_index* ix, Workspace& w, uint8_t* base, uint32_t qm,
                        uint32_t cm, uint32_t lm, uint64_t n_groups, uint32_t cand_cap,
                        bool outputs) {
  w.qcap = qm;
  w.cmax = cm;
  w.lmax = lm;
  w.ppad = round_up(std::max<uint32_t>(qm, 1), 256);
  w.cand_cap = cand_cap;
  const size_t tb = tile_bytes(ix->dt, ix->dpad);
  size_t off = 0;
  carve(&w.qrow, base, off, (size_t)qm * ix->dpad);
  carve(&w.qtiles, base, off, (size_t)round_up(qm, kTile) / kTile * tb);
  carve(&w.qscale, base, off, qm);
  carve(&w.qnorm, base, off, qm);
  // per-search inputs: [desc 4][k qm][clause_off qm+1][literal_off cm+1][terms lm]
  carve(&w.in, base, off, 4 + (size_t)qm + (qm + 1) + (cm + 1) + lm);
  if (w.in) {
    w.desc = w.in;
    w.k = w.desc + 4;
    w.clause_off = w.k + qm;
    w.literal_off = w.clause_off + qm + 1;
    w.terms = w.literal_off + cm + 1;
  }
  carve(&w.kp, base, off, qm);
  carve(&w.tau, base, off, qm);
  carve(&w.cnt, base, off, qm);
  carve(&w.smax, base, off, qm);
  carve(&w.hist, base, off, (size_t)qm * kHist);
  carve(&w.qlist, base, off, qm);
  carve(&w.qlist2, base, off, qm);
  carve(&w.ovf, base, off, qm);
  carve(&w.sel_cnt, base, off, qm);
  carve(&w.lit, base, off, (size_t)qm * kLits);
  carve(&w.linfo, base, off, qm);
  carve(&w.work, base, off, kXcds);
  carve(&w.hlo, base, off, qm);
  carve(&w.hinvw, base, off, qm);
  carve(&w.nmatch, base, off, qm);
  carve(&w.cand_key, base, off, (size_t)qm * cand_cap);
  carve(&w.skey, base, off, (size_t)qm * seed_row(ix));
  carve(&w.tsafe, base, off, qm);
  carve(&w.mw, base, off, (size_t)std::max<uint64_t>(n_groups, 1) * kWords * w.ppad);
  carve(&w.sel_key, base, off, (size_t)qm * ix->rmax);
  carve(&w.sel_slot, base, off, (size_t)qm * ix->rmax);
  if (ix->L) {
    carve(&w.dict, base, off, ix->batch_terms);
    carve(&w.bbits, base, off, (size_t)std::max<uint64_t>(n_groups, 1) * ix->batch_terms * kWords);
  }
  if (outputs) {
    carve(&w.slist, base, off, qm);
    carve(&w.srows, base, off, (size_t)qm * sparse_cap(ix));
  }
  if (outputs && ix->qbits) {
    carve(&w.qcode, base, off, (size_t)qm * (ix->qbits / 64));
    carve(&w.qhist, base, off, (size_t)qm * (ix->qbits + 1));
    carve(&w.qthr, base, off, qm);
    carve(&w.qneed, base, off, qm);
    carve(&w.qflag, base, off, qm);
    carve(&w.ntie, base, off, qm);
    carve(&w.surv, base, off, (size_t)qm * ix->scap);
    carve(&w.ties, base, off, (size_t)qm * ix->tcap);
    carve(&w.qkey, base, off, (size_t)qm * ix->scap);
  }
  if (outputs) {
    carve(&w.out_ids, base, off, (size_t)qm * ix->cfg.k_max);
    carve(&w.out_scores, base, off, (size_t)qm * ix->cfg.k_max);
    carve(&w.out_count, base, off, qm);
    carve(&w.out_nmatch, base, off, qm);
  }
  return off;
}

// The pinned twin of a workspace's input block, same layout.
void layout_host_inputs(Workspace& w, uint32_t* h_in) {
  w.h_in = h_in;
  w.h_desc = h_in;
  w.h_k = w.h_desc + 4;
  w.h_co = w.h_k + w.qcap;
  w.h_lo = w.h_co + w.qcap + 1;
  w.h_terms = w.h_lo + w.cmax + 1;
  w.h_dict = w.h_terms + w.lmax;
}

}  // namespace

namespace {

// Sign codes of n FP32 rows (`ld` floats apart) into their corpus slots,
// once the index has an encoding table.
hipError_t encode_rows(fr_index* ix, const float* rows, uint32_t ld, uint64_t n,
                       const uint32_t* slots, uint64_t slot_base) {
  if (!ix->quant_set || !n) return hipSuccess;
  SignArgs sa{};
  sa.rows = rows;
  sa.ld = ld;
  sa.n = n;
  sa.slots = slots;
  sa.slot_base = slot_base;
  sa.bin_off = ix->d_bin_off;
  sa.bin_dim = ix->d_bin_dim;
  sa.bin_sign = ix->d_bin_sign;
  sa.dim = ix->dim;
  sa.n_bits = ix->qbits;
  sa.codes = ix->codes;
  sa.corpus_layout = 1;
  return launch_sign_codes(sa, ix->stream);
}

// A document's terms into the index: bits of its slot in the per-term
// bitmaps (set, or cleared for a delete), or, with term lists, its list
// (a delete leaves the list: the live bit excludes the slot, and a later
// insert overwrites it).
hipError_t write_terms(fr_index* ix, const TermArgs& tm) {
  if (!ix->L) return launch_terms(tm, ix->stream);
  if (!tm.set) return hipSuccess;
  ListWriteArgs lw{};
  lw.off = tm.off;
  lw.terms = tm.terms;
  lw.slots = tm.slots;
  lw.slot_base = tm.slot_base;
  lw.n = tm.n;
  lw.tlist = ix->tlist;
  lw.tcnt = ix->tcnt;
  lw.L = ix->L;
  return launch_list_write(lw, ix->stream);
}

// With term lists, the bitmaps of the batch's dictionary terms, before a
// search's first mask pass.
hipError_t batch_bits(fr_index* ix, Workspace& w, uint32_t n_groups, hipStream_t s) {
  if (!ix->L) return hipSuccess;
  BatchBitsArgs bb{};
  bb.tlist = ix->tlist;
  bb.tcnt = ix->tcnt;
  bb.L = ix->L;
  bb.n_groups = n_groups;
  bb.dict = w.dict;
  bb.n_dict = w.n_dict;
  bb.bits = w.bbits;
  return launch_batch_bits(bb, s);
}

fr_status wait_all(fr_index* ix) {
  for (auto& w : ix->ws) {
    if (w.in_flight) {
      FR_HIP(hipEventSynchronize(w.fin));
      w.in_flight = false;
    }
  }
  if (ix->na_inflight) {
    FR_HIP(hipEventSynchronize(ix->na_done));
    ix->na_inflight = false;
  }
  FR_HIP(hipStreamSynchronize(ix->stream));
  ix->upd_pending = false;
  ix->ustage_pending = false;
  return FR_OK;
}

// Make the index stream wait (on the device) for every search still in
// flight: the workspaces' searches and the scratch-array search.
fr_status order_after_searches(fr_index* ix) {
  for (auto& w : ix->ws) {
    if (!w.in_flight) continue;
    if (hipEventQuery(w.fin) == hipSuccess) w.in_flight = false;
    else FR_HIP(hipStreamWaitEvent(ix->stream, w.fin, 0));
  }
  if (ix->na_inflight) {
    if (hipEventQuery(ix->na_done) == hipSuccess) ix->na_inflight = false;
    else FR_HIP(hipStreamWaitEvent(ix->stream, ix->na_done, 0));
  }
  return FR_OK;
}

// A search on stream s sees every update issued before it: s waits on the
// device for the last update (or, while s is being captured into a graph,
// the host waits, so that no outside event enters the capture).
fr_status order_after_update(fr_index* ix, hipStream_t s) {
  if (!ix->upd_pending) return FR_OK;
  if (hipEventQuery(ix->upd_done) == hipSuccess) {
    ix->upd_pending = false;
    return FR_OK;
  }
  if (s == ix->stream) return FR_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  FR_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    FR_HIP(hipEventSynchronize(ix->upd_done));
    ix->upd_pending = false;
    return FR_OK;
  }
  FR_HIP(hipStreamWaitEvent(s, ix->upd_done, 0));
  return FR_OK;
}

// The pinned update staging is refilled only once its last copies ran.
fr_status stage_wait(fr_index* ix) {
  if (ix->ustage_pending) {
    FR_HIP(hipEventSynchronize(ix->ustage_free));
    ix->ustage_pending = false;
  }
  return FR_OK;
}

// A document's term list as staged: as given, or, if longer than the
// staging holds, its distinct terms (at most the vocabulary, which fits);
// setting or clearing a bit twice is the same as once.
const uint32_t* doc_terms(const fr_index* ix, const uint32_t* t, uint64_t* len,
                          std::vector<uint32_t>& tmp) {
  if (*len <= ix->ustage_terms) return t;
  tmp.assign(t, t + *len);
  std::sort(tmp.begin(), tmp.end());
  tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
  *len = tmp.size();
  return tmp.data();
}

// Staged deletes h_dslots[0, m) with their term lists (h_doff, h_dterms):
// copy, clear live bits and slot ids, clear the listed term bits.
fr_status enqueue_deletes(fr_index* ix, uint64_t m, uint64_t nt) {
  if (!m) return FR_OK;
  FR_HIP(hipMemcpyAsync(ix->d_dslots, ix->h_dslots, m * 4, hipMemcpyHostToDevice, ix->stream));
  FR_HIP(hipMemcpyAsync(ix->d_doff, ix->h_doff, (m + 1) * 8, hipMemcpyHostToDevice, ix->stream));
  if (nt)
    FR_HIP(hipMemcpyAsync(ix->d_dterms, ix->h_dterms, nt * 4, hipMemcpyHostToDevice, ix->stream));
  FR_HIP(hipEventRecord(ix->ustage_free, ix->stream));
  ix->ustage_pending = true;
  LiveArgs la{};
  la.slots = ix->d_dslots;
  la.n = m;
  la.slot_ids = ix->slot_ids;
  la.live = ix->live;
  la.set = 0;
  FR_HIP(launch_live(la, ix->stream));
  TermArgs tm{};
  tm.off = ix->d_doff;
  tm.terms = ix->d_dterms;
  tm.slots = ix->d_dslots;
  tm.n = m;
  tm.bits = ix->bits;
  tm.vocab = ix->cfg.vocab;
  tm.set = 0;
  FR_HIP(write_terms(ix, tm));
  return FR_OK;
}

// Staged inserts (h_urows, h_uids, h_uslots, h_uoff, h_uterms) of m rows:
// copy, tile the rows into their slots, set term bits, ids and live bits.
fr_status enqueue_inserts(fr_index* ix, uint64_t m, uint64_t nt) {
  if (!m) return FR_OK;
  FR_HIP(hipMemcpyAsync(ix->d_urows, ix->h_urows, m * ix->dim * 4, hipMemcpyHostToDevice,
                        ix->stream));
  FR_HIP(hipMemcpyAsync(ix->d_uids, ix->h_uids, m * 4, hipMemcpyHostToDevice, ix->stream));
  FR_HIP(hipMemcpyAsync(ix->d_uslots, ix->h_uslots, m * 4, hipMemcpyHostToDevice, ix->stream));
  FR_HIP(hipMemcpyAsync(ix->d_uoff, ix->h_uoff, (m + 1) * 8, hipMemcpyHostToDevice, ix->stream));
  if (nt)
    FR_HIP(hipMemcpyAsync(ix->d_uterms, ix->h_uterms, nt * 4, hipMemcpyHostToDevice, ix->stream));
  FR_HIP(hipEventRecord(ix->ustage_free, ix->stream));
  ix->ustage_pending = true;
  TileRowsArgs ta{};
  ta.rows = ix->d_urows;
  ta.n = m;
  ta.dim = ix->dim;
  ta.dpad = ix->dpad;
  ta.dt = ix->dt;
  ta.slots = ix->d_uslots;
  ta.tiles = ix->tiles;
  ta.scale = ix->xscale;
  ta.master = ix->master;
  ta.norm_max = ix->norm_max;
  FR_HIP(launch_tile_rows(ta, ix->stream));
  FR_HIP(encode_rows(ix, ix->d_urows, ix->dim, m, ix->d_uslots, 0));
  TermArgs tm{};
  tm.off = ix->d_uoff;
  tm.terms = ix->d_uterms;
  tm.slots = ix->d_uslots;
  tm.n = m;
  tm.bits = ix->bits;
  tm.vocab = ix->cfg.vocab;
  tm.set = 1;
  FR_HIP(write_terms(ix, tm));
  LiveArgs la{};
  la.slots = ix->d_uslots;
  la.n = m;
  la.ids = ix->d_uids;
  la.slot_ids = ix->slot_ids;
  la.live = ix->live;
  la.set = 1;
  FR_HIP(launch_live(la, ix->stream));
  return FR_OK;
}

// Rewrite the host term store over live slots once half of it is garbage.
void compact_terms(fr_index* ix) {
  if (ix->t_garbage < (1u << 20) || ix->t_garbage * 2 < ix->t_arena.size()) return;
  std::vector<uint32_t> a;
  const uint64_t live = ix->t_arena.size() - ix->t_garbage;
  a.reserve(live + live / 4 + (1u << 22));
  for (uint64_t sl = 0; sl < ix->hwm; ++sl) {
    const uint32_t len = ix->t_len[sl];
    const uint64_t o = ix->t_off[sl];
    ix->t_off[sl] = a.size();
    a.insert(a.end(), ix->t_arena.begin() + o, ix->t_arena.begin() + o + len);
  }
  ix->t_arena.swap(a);
  ix->t_garbage = 0;
}

fr_status check_terms(const fr_index* ix, uint64_t n, const uint64_t* off, const uint32_t* terms) {
  if (n && (!off || (off[n] > off[0] && !terms)))
    return fail(FR_EINVAL, "term_off / terms missing");
  for (uint64_t i = 0; i < n; ++i) {
    if (off[i + 1] < off[i]) return fail(FR_EINVAL, "term_off must be non-decreasing");
    if (ix->L && off[i + 1] - off[i] > ix->L)
      return fail(FR_EINVAL, "a document has more terms than list_terms (" +
                                 std::to_string(ix->L) + ")");
  }
  for (uint64_t j = n ? off[0] : 0; j < (n ? off[n] : 0); ++j)
    if (terms[j] >= ix->cfg.vocab)
      return fail(FR_EINVAL, "term id " + std::to_string(terms[j]) + " >= vocab");
  return FR_OK;
}

// Finiteness of host rows, or of device rows via a kernel.
fr_status check_rows(fr_index* ix, const float* emb, uint64_t n, bool dev) {
  const uint64_t cnt = n * ix->dim;
  if (!cnt) return FR_OK;
  if (!emb) return fail(FR_EINVAL, "embeddings missing");
  if (!dev) {
    for (uint64_t i = 0; i < cnt; ++i)
      if (!std::isfinite(emb[i])) return fail(FR_EINVAL, "non-finite embedding value");
    return FR_OK;
  }
  FR_HIP(launch_fill_u32(ix->d_flag, 0u, 1, ix->stream));
  FR_HIP(launch_check_finite(emb, cnt, ix->d_flag, ix->stream));
  FR_HIP(hipMemcpyAsync(ix->h_flag, ix->d_flag, 4, hipMemcpyDeviceToHost, ix->stream));
  FR_HIP(hipStreamSynchronize(ix->stream));
  if (*ix->h_flag) return fail(FR_EINVAL, "non-finite embedding value");
  return FR_OK;
}

// Write rows [0, n) into slots (slots == null -> slot_base + i), with
// their term lists and ids.  Chunked through the pre-allocated staging.
fr_status write_docs(fr_index* ix, uint64_t n, const float* emb, const uint32_t* ids,
                     const uint64_t* off, const uint32_t* terms, const uint32_t* slots,
                     uint64_t slot_base, bool dev) {
  uint64_t r0 = 0;
  while (r0 < n) {
    uint64_t r1 = std::min(n, r0 + ix->stage_rows);
    while (r1 > r0 + 1 && off[r1] - off[r0] > ix->stage_terms) r1 = r0 + (r1 - r0) / 2;
    if (off[r1] - off[r0] > ix->stage_terms)
      return fail(FR_EUNSUPPORTED, "a document has more terms than the staging buffer");
    const uint64_t m = r1 - r0;
    const float* rows = emb + r0 * ix->dim;
    if (!dev) {
      FR_HIP(hipMemcpyAsync(ix->d_rows, rows, m * ix->dim * sizeof(float), hipMemcpyHostToDevice,
                            ix->stream));
      rows = ix->d_rows;
      FR_HIP(hipMemcpyAsync(ix->d_ids, ids + r0, m * 4, hipMemcpyHostToDevice, ix->stream));
    } else {
      FR_HIP(hipMemcpyAsync(ix->d_ids, ids + r0, m * 4, hipMemcpyDeviceToDevice, ix->stream));
    }
    std::vector<uint64_t> loc(m + 1);
    for (uint64_t i = 0; i <= m; ++i) loc[i] = off[r0 + i] - off[r0];
    FR_HIP(hipMemcpyAsync(ix->d_off, loc.data(), (m + 1) * 8, hipMemcpyHostToDevice, ix->stream));
    if (loc[m])
      FR_HIP(hipMemcpyAsync(ix->d_tl, terms + off[r0], loc[m] * 4, hipMemcpyHostToDevice,
                            ix->stream));
    if (slots)
      FR_HIP(hipMemcpyAsync(ix->d_slots, slots + r0, m * 4, hipMemcpyHostToDevice, ix->stream));
    TileRowsArgs ta{};
    ta.rows = rows;
    ta.n = m;
    ta.dim = ix->dim;
    ta.dpad = ix->dpad;
    ta.dt = ix->dt;
    ta.slots = slots ? ix->d_slots : nullptr;
    ta.slot_base = slot_base + r0;
    ta.tiles = ix->tiles;
    ta.scale = ix->xscale;
    ta.master = ix->master;
    ta.norm_max = ix->norm_max;
    FR_HIP(launch_tile_rows(ta, ix->stream));
    FR_HIP(encode_rows(ix, rows, ix->dim, m, ta.slots, ta.slot_base));
    TermArgs tm{};
    tm.off = ix->d_off;
    tm.terms = ix->d_tl;
    tm.slots = ta.slots;
    tm.slot_base = ta.slot_base;
    tm.n = m;
    tm.bits = ix->bits;
    tm.vocab = ix->cfg.vocab;
    tm.set = 1;
    FR_HIP(write_terms(ix, tm));
    LiveArgs la{};
    la.slots = ta.slots;
    la.slot_base = ta.slot_base;
    la.n = m;
    la.ids = ix->d_ids;
    la.slot_ids = ix->slot_ids;
    la.live = ix->live;
    la.set = 1;
    FR_HIP(launch_live(la, ix->stream));
    // the staging buffers are reused by the next chunk
    FR_HIP(hipStreamSynchronize(ix->stream));
    r0 = r1;
  }
  return FR_OK;
}

// Scan tiling for a batch: query blocks of 32 per wavefront (qb) and
// wavefronts per workgroup (nw), so qb*nw*32 queries share one pass over a
// group.  Default: the largest such tile that the batch fills (rounded up to
// 128 queries), preferring eight wavefronts (two per SIMD).
void pick_tiling(const fr_index* ix, uint32_t n_q, int* qb, int* nw) {
  const uint32_t want = round_up(std::max<uint32_t>(n_q, 1), 128);
  int bq = 1, bw = 4;
  uint32_t best = 0;
  for (int w : {4, 8})
    for (int c : {1, 2, 4}) {
      if (!scan_supported(ix->dt, ix->dpad, c, w)) continue;
      const uint32_t qt = 32u * c * w;
      if (qt > want && qt > 128) continue;
      if (qt > best || (qt == best && w > bw)) {
        best = qt;
        bq = c;
        bw = w;
      }
    }
  *qb = bq;
  *nw = bw;
}


// Buckets of the tuning table: ceil(log2 n_q), ceil(log2 of the largest
// selection size K'), and floor(-log2) of the median selectivity (0..20).
int q_bucket(uint32_t n_q) {
  int b = 0;
  while ((1u << b) < std::max<uint32_t>(n_q, 1) && b < 31) ++b;
  return b;
}
uint32_t sel_size(const fr_index* ix, uint32_t k) {
  if (ix->dt == kF32 || !k) return k;
  return std::max(k, std::min(ix->r, std::max(ix->r_min, 4u * k)));
}
int sel_bucket(double sel) {
  if (!(sel > 0.0)) return 20;
  return (int)std::min(20.0, std::max(0.0, std::floor(-std::log2(sel))));
}

// Tiling and strategy of one search: a pinned choice (fr_set_tiling /
// fr_set_strategy), else the tuning table's entry for the batch's Q and K'
// buckets (of several selectivity buckets, the one nearest the last
// measured), else the per-batch defaults.
struct Choice {
  int qb, nw, gpi;
  uint32_t strat;
  int source;   // 0 defaults, 1 pinned, 2 tuning table
};
Choice choose(const fr_index* ix, uint32_t n_q, const uint32_t* k, uint32_t n_groups) {
  Choice c{1, 4, 0, ix->strat, 0};
  uint32_t kmax = 0;
  for (uint32_t q = 0; q < n_q; ++q) kmax = std::max(kmax, sel_size(ix, k[q]));
  const int qk = q_bucket(n_q), kk = q_bucket(kmax);
  const fr_index::Tuned* hit = nullptr;
  int best_d = 1 << 30;
  for (const auto& e : ix->tuned) {
    if (std::get<0>(e.first) != qk || std::get<1>(e.first) != kk) continue;
    const int d = ix->last_sel < 0 ? 0 : std::abs(std::get<2>(e.first) - ix->last_sel);
    if (d < best_d) {
      best_d = d;
      hit = &e.second;
    }
  }
  if (ix->qb && ix->nw) {
    c.qb = ix->qb;
    c.nw = ix->nw;
    c.gpi = ix->gpi;
    c.source = 1;
  } else if (hit) {
    c.qb = hit->qb;
    c.nw = hit->nw;
    c.gpi = hit->gpi;
    if (!ix->strat_pinned) c.strat = hit->strat;
    c.source = 2;
  } else {
    pick_tiling(ix, n_q, &c.qb, &c.nw);
    c.gpi = ix->gpi;
  }
  if (!c.gpi) {
    const uint64_t qtiles = (n_q + 32u * c.qb * c.nw - 1) / (32u * c.qb * c.nw);
    const uint64_t g = ((uint64_t)n_groups * qtiles + ix->n_wg) / (2ull * ix->n_wg);
    c.gpi = (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 16));
  }
  return c;
}

// Per-query state of a search (thresholds, histograms, lists, literal
// tables) for the batch staged in workspace w.
PrepArgs prep_args(const fr_index* ix, Workspace& w) {
  PrepArgs pa{};
  pa.max_q = w.qcap;
  pa.n_dev = w.desc;
  pa.k = w.k;
  pa.kp = w.kp;
  pa.dt = ix->dt;
  pa.rescore_r = ix->r;
  pa.rescore_min = ix->r_min;
  pa.qnorm = w.qnorm;
  pa.norm_max = ix->norm_max;
  pa.tau = w.tau;
  pa.tsafe = w.tsafe;
  pa.cnt = w.cnt;
  pa.smax = w.smax;
  pa.hist = w.hist;
  pa.hlo = w.hlo;
  pa.hinvw = w.hinvw;
  pa.nmatch = w.nmatch;
  pa.qlist = w.qlist;
  pa.n_list = w.desc + 1;
  pa.n_list2 = w.desc + 2;
  pa.work = w.work;
  pa.ovf = w.ovf;
  pa.clause_off = w.clause_off;
  pa.literal_off = w.literal_off;
  pa.terms = w.terms;
  pa.lit = w.lit;
  pa.linfo = w.linfo;
  return pa;
}

// Predicate masks of the first pass (every query of the batch) into w.mw,
// counting each query's matches.
MaskWordArgs mask_args(const fr_index* ix, Workspace& w, uint32_t n_groups) {
  MaskWordArgs ma{};
  ma.qlist = w.qlist;
  ma.n_list = w.desc + 1;
  ma.max_list = w.qcap;
  ma.ppad = w.ppad;
  ma.n_groups = n_groups;
  // groups per thread: about eight blocks of 32 of the batch's queries per
  // compute unit (blocks past the batch exit at once)
  const uint64_t qblocks = (std::max<uint32_t>(w.h_desc[0], 1u) + 31u) / 32u;
  ma.gpt = std::max<uint32_t>(1, std::min<uint32_t>(16, (uint32_t)(((uint64_t)n_groups * qblocks) >> 11)));
  ma.live = ix->live;
  ma.bits = ix->L ? w.bbits : ix->bits;
  ma.vocab = ix->L ? w.n_dict : ix->cfg.vocab;
  ma.lit = w.lit;
  ma.linfo = w.linfo;
  ma.clause_off = w.clause_off;
  ma.literal_off = w.literal_off;
  ma.terms = w.terms;
  ma.mw = w.mw;
  ma.nmatch = w.nmatch;
  ma.count_matches = 1;
  ma.run_if = nullptr;   // the first pass always runs
  return ma;
}

// Tiles per scan work item.  Work items are (tile range, query tile) pairs
// taken from per-XCD queues, the query tiles of one range together on one
// XCD.  When each XCD's workgroups can hold whole ranges for all query tiles
// at once, the corpus is cut into as many equal ranges as fit, so that every
// workgroup takes one item of the same size: whole 1024-document groups (the
// tuned groups per item) would leave up to a group's worth of work per
// workgroup idle at the end (1M documents are 977 groups for 256
// workgroups).  Otherwise the tuned groups per item.  A multiple of 4, the
// largest number of tiles per ring slot.
uint32_t scan_tiles_per_item(const fr_index* ix, const Workspace& w, const Choice& ch,
                             uint32_t n_groups) {
  const uint64_t n_tiles = (uint64_t)n_groups * (kGroup / kTile);
  const uint64_t qt = (std::max<uint32_t>(w.h_desc[0], 1u) + 32u * ch.qb * ch.nw - 1) /
                      (32u * ch.qb * ch.nw);
  const uint64_t wg_xcd = std::max<uint64_t>((uint64_t)ix->n_wg / kXcds, 1);
  uint64_t tpi = (uint64_t)std::max(ch.gpi, 1) * (kGroup / kTile);
  if (qt <= wg_xcd) {
    const uint64_t ranges = (uint64_t)kXcds * (wg_xcd / qt);
    tpi = (n_tiles + ranges - 1) / ranges;
  }
  tpi = (tpi + 3) / 4 * 4;
  return (uint32_t)std::max<uint64_t>(tpi, 4);
}

fr_status enqueue_search(fr_index* ix, Workspace& w, hipStream_t s, const Choice& ch,
                         uint32_t n_groups, bool timing, const float* qsrc, uint32_t* o_ids,
                         float* o_scores, uint32_t* o_count, unsigned long long* o_nmatch) {
  // query rows: the workspace's padded copy (host queries), or the caller's
  // device rows, of which the kernel then writes the padded copy that the
  // FP32 rescoring reads
  TileRowsArgs ta{};
  const bool in_place = qsrc != w.qrow;
  ta.rows = qsrc;
  ta.n = w.qcap;
  ta.n_dev = w.desc;
  ta.dim = in_place ? ix->dim : ix->dpad;
  ta.dpad = ix->dpad;
  ta.master = (in_place && ix->dt != kF32) ? w.qrow : nullptr;
  ta.dt = ix->dt;
  ta.tiles = w.qtiles;
  ta.scale = w.qscale;
  ta.norm = w.qnorm;
  FR_HIP(launch_query_prep(ta, prep_args(ix, w), s));
  FR_HIP(batch_bits(ix, w, n_groups, s));
  const MaskWordArgs ma = mask_args(ix, w, n_groups);
  FR_HIP(launch_mask_words(ma, s));

  SelectArgs se{};
  se.qlist = w.qlist;
  se.n_list = w.desc + 1;
  se.max_list = w.qcap;
  se.final_pass = 0;
  se.kp = w.kp;
  se.tau = w.tau;
  se.cnt = w.cnt;
  se.smax = w.smax;
  se.hist = w.hist;
  se.hlo = w.hlo;
  se.hinvw = w.hinvw;
  se.qlist2 = w.qlist2;
  se.n_list2 = w.desc + 2;
  se.work = w.work;
  se.qnorm = w.qnorm;
  se.norm_max = ix->norm_max;
  se.cand_key = w.cand_key;
  se.slot_ids = ix->slot_ids;
  se.cap = w.cand_cap;
  se.sel_key = w.sel_key;
  se.sel_slot = w.sel_slot;
  se.sel_cnt = w.sel_cnt;
  se.rmax = ix->rmax;
  se.ovf = w.ovf;
  se.tsafe = w.tsafe;
  se.write_out = ix->dt == kF32;
  se.k = w.k;
  se.k_max = ix->cfg.k_max;
  se.out_ids = o_ids;
  se.out_scores = o_scores;
  se.out_count = o_count;
  se.nmatch = w.nmatch;
  se.out_nmatch = o_nmatch;

  // Sparse routing (strategy level L > 0): queries with at most
  // n_live * 2^(L-11) matches leave the scan's list; their matching rows are
  // listed from this pass's masks (stored at position = query) and scored
  // one by one in FP32, and the exact selection takes their top K'.  The
  // masks are then laid out again for the scan's shorter list (a pass that
  // does nothing when no query was routed).
  const uint32_t lvl = (ch.strat & kStratSparseMask) >> kStratSparseShift;
  if (lvl && w.srows) {
    const uint32_t rcap = sparse_cap(ix);
    const uint32_t limit = (uint32_t)std::min<double>(
        std::ldexp((double)ix->n_live, (int)lvl - 11), (double)rcap);
    RouteArgs ra{};
    ra.max_q = w.qcap;
    ra.n_dev = w.desc;
    ra.nmatch = w.nmatch;
    ra.kp = w.kp;
    ra.cap_by_kp = ix->dt != kF32;
    ra.limit = limit;
    ra.qlist = w.qlist;
    ra.n_list = w.desc + 1;
    ra.slist = w.slist;
    ra.n_slist = w.desc + 3;
    FR_HIP(launch_route(ra, s));
    SparseRowsArgs sr{};
    sr.max_q = w.qcap;
    sr.slist = w.slist;
    sr.n_slist = w.desc + 3;
    sr.mw = w.mw;
    sr.ppad = ma.ppad;
    sr.n_groups = n_groups;
    sr.gpb = 16;
    sr.cnt = w.cnt;
    sr.rows = w.srows;
    sr.cap = rcap;
    FR_HIP(launch_sparse_rows(sr, s));
    RowDotArgs rd{};
    rd.max_q = w.qcap;
    rd.n_dev = w.desc;
    rd.qlist = w.slist;
    rd.n_list = w.desc + 3;
    rd.cnt = w.cnt;
    rd.rows = w.srows;
    rd.stride = rcap;
    rd.max_cnt = limit;
    rd.master = ix->master;
    rd.tiles = ix->master ? nullptr : ix->tiles;
    rd.dpad = ix->dpad;
    rd.qrows = qsrc;
    rd.q_ld = in_place ? ix->dim : ix->dpad;
    rd.dim = ix->dim;
    rd.key = w.cand_key;
    rd.key_stride = w.cand_cap;
    rd.hist = w.hist;
    rd.hlo = w.hlo;
    rd.hinvw = w.hinvw;
    FR_HIP(launch_row_dots(rd, s));
    SelectArgs ss = se;
    ss.qlist = w.slist;
    ss.n_list = w.desc + 3;
    ss.final_pass = 1;
    FR_HIP(launch_select(ss, s));
    MaskWordArgs mr = ma;
    mr.count_matches = 0;
    mr.run_if = w.desc + 3;
    FR_HIP(launch_mask_words(mr, s));
  }

  SeedArgs sd{};
  sd.qlist = w.qlist;
  sd.n_list = w.desc + 1;
  sd.max_list = w.qcap;
  sd.kp = w.kp;
  sd.tiles = ix->tiles;
  sd.xscale = ix->xscale;
  sd.qtiles = w.qtiles;
  sd.qscale = w.qscale;
  sd.qnorm = w.qnorm;
  sd.norm_max = ix->norm_max;
  sd.mw = w.mw;
  sd.ppad = ma.ppad;
  sd.n_groups = std::min(n_groups, ix->seed_groups);
  sd.dim = ix->dim;
  sd.skey = w.skey;
  sd.row = seed_row(ix);
  sd.nmatch = w.nmatch;
  sd.tau = w.tau;
  sd.tsafe = w.tsafe;
  sd.strategy = ch.strat;
  sd.hlo = w.hlo;
  sd.hinvw = w.hinvw;
  FR_HIP(launch_seed(sd, ix->dt, ix->dpad, s));

  ScanArgs sa{};
  sa.tiles = ix->tiles;
  sa.xscale = ix->xscale;
  sa.live = ix->live;
  sa.bits = ix->L ? w.bbits : ix->bits;
  sa.vocab = ix->L ? w.n_dict : ix->cfg.vocab;
  sa.n_groups = n_groups;
  sa.qtiles = w.qtiles;
  sa.qscale = w.qscale;
  sa.qlist = w.qlist;
  sa.n_list = w.desc + 1;
  sa.kp = w.kp;
  sa.tau = w.tau;
  sa.cnt = w.cnt;
  sa.smax = w.smax;
  sa.hist = w.hist;
  sa.hlo = w.hlo;
  sa.hinvw = w.hinvw;
  sa.cand_key = w.cand_key;
  sa.cap = w.cand_cap;
  sa.work = w.work;
  sa.tpi = scan_tiles_per_item(ix, w, ch, n_groups);
  sa.strategy = ch.strat;
  sa.mw = w.mw;
  sa.ppad = ma.ppad;
  if (timing) FR_HIP(hipEventRecord(w.e_scan0, s));
  FR_HIP(launch_scan(sa, ix->dt, ix->dpad, ch.qb, ch.nw, ix->n_wg, s));
  if (timing) FR_HIP(hipEventRecord(w.e_scan1, s));
  FR_HIP(launch_select(se, s));

  // second pass for the queries the first could not answer (an empty list
  // when there are none)
  MaskWordArgs mb = ma;
  mb.qlist = w.qlist2;
  mb.n_list = w.desc + 2;
  mb.count_matches = 0;
  FR_HIP(launch_mask_words(mb, s));
  ScanArgs sb = sa;
  sb.qlist = w.qlist2;
  sb.n_list = w.desc + 2;
  FR_HIP(launch_scan(sb, ix->dt, ix->dpad, ch.qb, ch.nw, ix->n_wg, s));
  SelectArgs sf = se;
  sf.qlist = w.qlist2;
  sf.n_list = w.desc + 2;
  sf.final_pass = 1;
  FR_HIP(launch_select(sf, s));

  if (ix->dt != kF32) {
    RescoreArgs rs{};
    rs.max_q = w.qcap;
    rs.n_dev = w.desc;
    rs.ovf = w.ovf;
    rs.master = ix->master;
    rs.qrows = w.qrow;
    rs.dpad = ix->dpad;
    rs.sel_key = w.sel_key;
    rs.sel_slot = w.sel_slot;
    rs.sel_cnt = w.sel_cnt;
    rs.rmax = ix->rmax;
    rs.k = w.k;
    rs.k_max = ix->cfg.k_max;
    rs.out_ids = o_ids;
    rs.out_scores = o_scores;
    rs.out_count = o_count;
    rs.nmatch = w.nmatch;
    rs.out_nmatch = o_nmatch;
    FR_HIP(launch_rescore(rs, s));
  }
  return FR_OK;
}

// Sign-code pre-selection search (FR_PRESELECT): query prep and masks as for
// a plain search, query codes, the histogram pass, the per-query cut, the
// collect pass, the lowest-id ties, FP32 scores of the survivors, and the
// exact selection of their top K.  `max_qk` is the batch's largest quantK.
fr_status enqueue_preselect(fr_index* ix, Workspace& w, hipStream_t s, uint32_t n_groups,
                            uint32_t max_qk, bool timing, const float* qsrc, uint32_t* o_ids,
                            float* o_scores, uint32_t* o_count, unsigned long long* o_nm) {
  TileRowsArgs ta{};
  const bool in_place = qsrc != w.qrow;
  ta.rows = qsrc;
  ta.n = w.qcap;
  ta.n_dev = w.desc;
  ta.dim = in_place ? ix->dim : ix->dpad;
  ta.dpad = ix->dpad;
  ta.dt = ix->dt;
  ta.tiles = w.qtiles;
  ta.scale = w.qscale;
  ta.norm = w.qnorm;
  FR_HIP(launch_query_prep(ta, prep_args(ix, w), s));
  const uint32_t q_ld = in_place ? ix->dim : ix->dpad;
  SignArgs qa{};
  qa.rows = qsrc;
  qa.ld = q_ld;
  qa.n = w.qcap;
  qa.n_dev = w.desc;
  qa.bin_off = ix->d_bin_off;
  qa.bin_dim = ix->d_bin_dim;
  qa.bin_sign = ix->d_bin_sign;
  qa.dim = ix->dim;
  qa.n_bits = ix->qbits;
  qa.codes = w.qcode;
  FR_HIP(launch_sign_codes(qa, s));
  FR_HIP(batch_bits(ix, w, n_groups, s));
  const MaskWordArgs ma = mask_args(ix, w, n_groups);
  FR_HIP(launch_mask_words(ma, s));
  FR_HIP(launch_fill_u32(w.qhist, 0u, (uint64_t)w.qcap * (ix->qbits + 1), s));

  QuantArgs qs{};
  qs.codes = ix->codes;
  qs.qcode = w.qcode;
  qs.mw = w.mw;
  qs.ppad = ma.ppad;
  qs.n_slices = n_groups * (uint32_t)kWords;
  qs.max_q = w.qcap;
  qs.n_dev = w.desc;
  qs.n_bits = ix->qbits;
  // about four blocks per compute unit over the batch's query blocks
  const uint32_t qblocks = (w.qcap + kQuantQB - 1) / kQuantQB;
  const uint32_t xblocks = std::max<uint32_t>(1, (uint32_t)(4 * ix->n_cu) / qblocks);
  qs.spb = std::max<uint32_t>(4, round_up((qs.n_slices + xblocks - 1) / xblocks, 4));
  qs.hist = w.qhist;
  qs.thr = w.qthr;
  qs.flag = w.qflag;
  qs.cnt = w.cnt;
  qs.surv = w.surv;
  qs.scap = ix->scap;
  qs.ntie = w.ntie;
  qs.ties = w.ties;
  qs.tcap = ix->tcap;
  if (timing) FR_HIP(hipEventRecord(w.e_scan0, s));
  FR_HIP(launch_quant_hist(qs, s));

  QuantSelectArgs qc{};
  qc.max_q = w.qcap;
  qc.n_dev = w.desc;
  qc.k = w.k;
  qc.factor = ix->qfactor;
  qc.n_bits = ix->qbits;
  qc.hist = w.qhist;
  qc.thr = w.qthr;
  qc.need = w.qneed;
  qc.flag = w.qflag;
  qc.cnt = w.cnt;
  qc.ntie = w.ntie;
  qc.ties = w.ties;
  qc.surv = w.surv;
  qc.scap = ix->scap;
  qc.tcap = ix->tcap;
  qc.slot_ids = ix->slot_ids;
  qc.tau = w.tau;
  qc.hinvw = w.hinvw;
  qc.tsafe = w.tsafe;
  qc.ovf = w.ovf;
  FR_HIP(launch_quant_cut(qc, s));
  FR_HIP(launch_quant_collect(qs, s));
  if (timing) FR_HIP(hipEventRecord(w.e_scan1, s));
  FR_HIP(launch_quant_ties(qc, s));

  RowDotArgs qd{};
  qd.max_q = w.qcap;
  qd.n_dev = w.desc;
  qd.cnt = w.cnt;
  qd.rows = w.surv;
  qd.stride = ix->scap;
  qd.max_cnt = max_qk;
  qd.master = ix->master;
  qd.dpad = ix->dpad;
  qd.qrows = qsrc;
  qd.q_ld = q_ld;
  qd.dim = ix->dim;
  qd.key = w.qkey;
  qd.key_stride = ix->scap;
  qd.hist = nullptr;   // the selection sorts every survivor (no cut)
  qd.hlo = nullptr;
  qd.hinvw = nullptr;
  FR_HIP(launch_row_dots(qd, s));

  SelectArgs se{};
  se.qlist = w.qlist;
  se.n_list = w.desc + 1;
  se.max_list = w.qcap;
  se.final_pass = 1;
  se.kp = w.k;
  se.tau = w.tau;
  se.cnt = w.cnt;
  se.smax = w.smax;
  se.hist = w.hist;
  se.hlo = w.hlo;
  se.hinvw = w.hinvw;
  se.qlist2 = w.qlist2;
  se.n_list2 = w.desc + 2;
  se.work = w.work;
  se.qnorm = w.qnorm;
  se.norm_max = ix->norm_max;
  se.cand_key = w.qkey;
  se.slot_ids = ix->slot_ids;
  se.cap = ix->scap;
  se.sel_key = w.sel_key;
  se.sel_slot = w.sel_slot;
  se.sel_cnt = w.sel_cnt;
  se.rmax = ix->rmax;
  se.ovf = w.ovf;
  se.tsafe = w.tsafe;
  se.write_out = 1;
  se.k = w.k;
  se.k_max = ix->cfg.k_max;
  se.out_ids = o_ids;
  se.out_scores = o_scores;
  se.out_count = o_count;
  se.nmatch = w.nmatch;
  se.out_nmatch = o_nm;
  FR_HIP(launch_select(se, s));
  return FR_OK;
}

// Pick the timing-ring slot of a call and remember it in the history.
void ring_slot(fr_index* ix, Workspace& w) {
  const int slot = (int)(w.n_calls % Workspace::kRing);
  w.e_scan0 = w.r0[slot];
  w.e_scan1 = w.r1[slot];
  w.e_start = w.r3[slot];
  w.e_end = w.r2[slot];
  w.n_calls += 1;
  ix->history.emplace_back((uint32_t)(&w - ix->ws.data()), (uint32_t)slot);
  if (ix->history.size() > (size_t)Workspace::kRing)
    ix->history.erase(ix->history.begin(),
                      ix->history.begin() + (ix->history.size() - Workspace::kRing));
}

void drop_graph(Workspace& w) {
  if (w.gexec) (void)hipGraphExecDestroy(w.gexec);
  if (w.graph) (void)hipGraphDestroy(w.graph);
  w.gexec = nullptr;
  w.graph = nullptr;
}

fr_status validate_cnf(const fr_index* ix, uint32_t n_q, const fr_cnf_batch* cnf, uint32_t* n_c,
                       uint32_t* n_l) {
  if (!cnf) return fail(FR_EINVAL, "cnf batch missing");
  if (cnf->n_queries != n_q) return fail(FR_EINVAL, "cnf->n_queries != n_q");
  if (!cnf->clause_off) return fail(FR_EINVAL, "clause_off missing");
  if (cnf->clause_off[0] != 0) return fail(FR_EINVAL, "clause_off[0] must be 0");
  for (uint32_t q = 0; q < n_q; ++q)
    if (cnf->clause_off[q + 1] < cnf->clause_off[q])
      return fail(FR_EINVAL, "clause_off must be non-decreasing");
  const uint32_t c = cnf->clause_off[n_q];
  if (c > ix->cmax) return fail(FR_EINVAL, "more clauses than max_clauses");
  if (c && !cnf->literal_off) return fail(FR_EINVAL, "literal_off missing");
  if (c && cnf->literal_off[0] != 0) return fail(FR_EINVAL, "literal_off[0] must be 0");
  for (uint32_t i = 0; i < c; ++i)
    if (cnf->literal_off[i + 1] < cnf->literal_off[i])
      return fail(FR_EINVAL, "literal_off must be non-decreasing");
  const uint32_t l = c ? cnf->literal_off[c] : 0;
  if (l > ix->lmax) return fail(FR_EINVAL, "more literals than max_literals");
  if (l && !cnf->terms) return fail(FR_EINVAL, "terms missing");
  for (uint32_t i = 0; i < l; ++i)
    if (cnf->terms[i] >= ix->cfg.vocab)
      return fail(FR_EINVAL, "literal term " + std::to_string(cnf->terms[i]) + " >= vocab");
  *n_c = c;
  *n_l = l;
  return FR_OK;
}

// Copy the CNF batch into a workspace's pinned input block, then the block
// (descriptor, K values and CNF, up to the last term used) to the device in
// one copy.
fr_status stage_inputs(fr_index* ix, Workspace& w, hipStream_t s, uint32_t n_q,
                       const fr_cnf_batch* cnf, uint32_t n_c, uint32_t n_l) {
  std::memcpy(w.h_co, cnf->clause_off, (n_q + 1) * 4);
  if (n_c) std::memcpy(w.h_lo, cnf->literal_off, (n_c + 1) * 4);
  else w.h_lo[0] = 0;
  if (ix->L) {
    // term lists: the batch's distinct terms, sorted, and the literals as
    // their indices (the bitmaps are built for these terms only)
    std::vector<uint32_t> u(cnf->terms, cnf->terms + n_l);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    if (u.size() > ix->batch_terms)
      return fail(FR_EINVAL, "the batch has " + std::to_string(u.size()) +
                                 " distinct terms, more than batch_terms (" +
                                 std::to_string(ix->batch_terms) + ")");
    for (uint32_t i = 0; i < n_l; ++i)
      w.h_terms[i] = (uint32_t)(std::lower_bound(u.begin(), u.end(), cnf->terms[i]) - u.begin());
    if (!u.empty()) std::memcpy(w.h_dict, u.data(), u.size() * 4);
    w.n_dict = (uint32_t)u.size();
    if (w.n_dict)
      FR_HIP(hipMemcpyAsync(w.dict, w.h_dict, w.n_dict * 4, hipMemcpyHostToDevice, s));
  } else if (n_l) {
    std::memcpy(w.h_terms, cnf->terms, n_l * 4);
  }
  const size_t words = (size_t)(w.h_terms - w.h_in) + n_l;
  FR_HIP(hipMemcpyAsync(w.in, w.h_in, words * 4, hipMemcpyHostToDevice, s));
  return FR_OK;
}

Workspace* acquire_ws(fr_index* ix, bool nowait, fr_status* st) {
  const size_t n = ix->ws.size();
  // prefer a workspace that is already free
  for (size_t i = 0; i < n; ++i) {
    Workspace& w = ix->ws[(ix->next_ws + i) % n];
    if (!w.in_flight || hipEventQuery(w.fin) == hipSuccess) {
      w.in_flight = false;
      ix->next_ws = (ix->next_ws + i + 1) % n;
      *st = FR_OK;
      return &w;
    }
  }
  if (nowait) {
    *st = fail(FR_EBUSY, "all workspaces are in use");
    return nullptr;
  }
  Workspace& w = ix->ws[ix->next_ws];
  ix->next_ws = (ix->next_ws + 1) % n;
  if (hipEventSynchronize(w.fin) != hipSuccess) {
    ix->failed = true;
    *st = fail(FR_EDEVICE, "hipEventSynchronize failed");
    return nullptr;
  }
  w.in_flight = false;
  *st = FR_OK;
  return &w;
}

}  // namespace

namespace fr {

fr_status set_error(fr_status s, const std::string& msg) { return fail(s, msg); }

fr_status index_shape(fr_index* ix, IndexShape* out) {
  if (!ix || !out) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  out->dim = ix->dim;
  out->vocab = ix->cfg.vocab;
  out->k_max = ix->cfg.k_max;
  out->max_batch = ix->qmax;
  out->max_clauses = ix->cmax;
  out->max_literals = ix->lmax;
  out->n_workspaces = (uint32_t)ix->ws.size();
  out->batch_terms = ix->batch_terms;
  out->device = ix->cfg.device;
  return FR_OK;
}

}  // namespace fr

extern "C" {

const char* fr_last_error(void) { return g_err.c_str(); }

fr_status fr_create(const fr_config* cfg, fr_index** out) {
  if (!cfg || !out) return fail(FR_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->dim < 1 || cfg->dim > 256) return fail(FR_EUNSUPPORTED, "dim must be 1..256");
  if (cfg->list_terms > 4096) return fail(FR_EINVAL, "list_terms must be 0..4096");
  if (cfg->batch_terms > (uint32_t)kBatchTermsMax)
    return fail(FR_EINVAL, "batch_terms must be 0..1024");
  if (cfg->vocab < 1 || cfg->vocab > (cfg->list_terms ? (1u << 31) : (1u << 20)))
    return fail(FR_EINVAL, "vocab must be 1..2^20 (1..2^31 with list_terms)");
  if (cfg->k_max < 1 || cfg->k_max > (uint32_t)kMaxR) return fail(FR_EINVAL, "k_max must be 1..4096");
  if (cfg->capacity < 1 || cfg->capacity > (1ull << 32) - kGroup)
    return fail(FR_EINVAL, "capacity must be 1..2^32-1024");
  if (cfg->dtype != FR_F32 && cfg->dtype != FR_BF16 && cfg->dtype != FR_FP8_E4M3)
    return fail(FR_EINVAL, "unknown dtype");
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || cfg->device < 0 || cfg->device >= n_dev)
    return fail(FR_EDEVICE, "no such HIP device");
  std::unique_ptr<fr_index> holder(new fr_index());
  fr_index* ix = holder.get();
  ix->cfg = *cfg;
  ix->dt = (int)cfg->dtype;
  ix->dim = cfg->dim;
  ix->dpad = round_up(cfg->dim, 64);
  ix->cap = (cfg->capacity + kGroup - 1) / kGroup * kGroup;
  ix->r = cfg->rescore_r ? cfg->rescore_r : (uint32_t)kMaxR;
  if (ix->dt != kF32 && (ix->r < cfg->k_max || ix->r > (uint32_t)kMaxR))
    return fail(FR_EINVAL, "rescore_r must be k_max..4096");
  ix->r_min = cfg->rescore_min ? std::min(cfg->rescore_min, ix->r) : ix->r;
  ix->rmax = ix->dt == kF32 ? cfg->k_max : ix->r;
  ix->qmax = cfg->max_batch ? cfg->max_batch : 1024;
  ix->seed_groups = ix->dt == kF32 ? kSeedGroupsF32 : kSeedGroupsLow;
  // default strategy: speculative start, no threshold refresh during the
  // scan (with the selection's own bucket cut the refresh costs more than
  // the candidates it saves on the measured workloads)
  ix->strat = FR_STRAT_NO_REFRESH;
  if (ix->qmax > 65536) return fail(FR_EINVAL, "max_batch must be <= 65536");
  ix->cmax = cfg->max_clauses ? cfg->max_clauses : 8 * ix->qmax;
  ix->lmax = cfg->max_literals ? cfg->max_literals : 32 * ix->qmax;
  ix->cand_cap = cfg->cand_cap ? cfg->cand_cap : std::max<uint32_t>(16384, 16 * ix->rmax);
  if (ix->cand_cap < ix->rmax) return fail(FR_EINVAL, "cand_cap must be >= the selection size");
  if (!scan_supported(ix->dt, ix->dpad, 1, 4))
    return fail(FR_EUNSUPPORTED, "no scan kernel for this dtype/dim");
  ix->L = cfg->list_terms;
  ix->batch_terms = ix->L ? (cfg->batch_terms ? cfg->batch_terms : (uint32_t)kBatchTermsMax) : 0;
  ix->qbits = cfg->quant_bits;
  if (ix->qbits && ix->qbits != 64 && ix->qbits != 128 && ix->qbits != 256 && ix->qbits != 512)
    return fail(FR_EINVAL, "quant_bits must be 0, 64, 128, 256 or 512");
  ix->qfactor = cfg->quant_factor ? cfg->quant_factor : 200;
  if (ix->qbits) {
    ix->scap = (uint32_t)std::min<uint64_t>((uint64_t)ix->qfactor * cfg->k_max, kQuantMaxK);
    ix->tcap = std::max<uint32_t>(ix->scap, 16384);
    ix->bin_cap = (uint64_t)ix->qbits * ix->dpad;
  }
  std::vector<void*>& D = ix->dev_owned;
  std::vector<void*>& H = ix->host_owned;
  auto cleanup = [&]() {
    for (void* p : D) (void)hipFree(p);
    for (void* p : H) (void)hipHostFree(p);
    D.clear();
    H.clear();
  };
#define FR_ALLOC(expr)                                                    \
  do {                                                                    \
    if ((expr) != hipSuccess) {                                           \
      cleanup();                                                          \
      return fail(FR_ENOMEM, std::string("allocation failed: ") + #expr); \
    }                                                                     \
  } while (0)
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(FR_EDEVICE, "hipSetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess)
    return fail(FR_EDEVICE, "hipGetDeviceProperties failed");
  ix->n_cu = prop.multiProcessorCount;
  {
    size_t i = 0;
    for (; i + 1 < sizeof ix->arch && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
      ix->arch[i] = prop.gcnArchName[i];
    ix->arch[i] = 0;
  }
  ix->n_wg = std::max(kXcds, ix->n_cu / kXcds * kXcds);
  if (hipStreamCreateWithFlags(&ix->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FR_EDEVICE, "hipStreamCreate failed");

  const uint64_t cap = ix->cap;
  const size_t tb = tile_bytes(ix->dt, ix->dpad);
  FR_ALLOC(dalloc(&ix->tiles, cap / kTile * tb, D));
  if (ix->dt == kFP8) FR_ALLOC(dalloc(&ix->xscale, cap, D));
  if (ix->dt != kF32 || ix->qbits) FR_ALLOC(dalloc(&ix->master, cap * ix->dpad, D));
  if (ix->qbits) {
    FR_ALLOC(dalloc(&ix->codes, cap * (ix->qbits / 64), D));
    FR_ALLOC(dalloc(&ix->d_bin_off, ix->qbits + 1, D));
    FR_ALLOC(dalloc(&ix->d_bin_dim, ix->bin_cap, D));
    FR_ALLOC(dalloc(&ix->d_bin_sign, ix->bin_cap, D));
  }
  FR_ALLOC(dalloc(&ix->slot_ids, cap, D));
  FR_ALLOC(dalloc(&ix->live, cap / 64, D));
  if (ix->L) {
    FR_ALLOC(dalloc(&ix->tlist, cap * ix->L, D));
    FR_ALLOC(dalloc(&ix->tcnt, cap, D));
  } else {
    FR_ALLOC(dalloc(&ix->bits, cap / kGroup * (uint64_t)cfg->vocab * kWords, D));
  }
  FR_ALLOC(dalloc(&ix->norm_max, 1, D));
  FR_ALLOC(dalloc(&ix->d_flag, 1, D));
  ix->stage_rows = std::min<uint64_t>(cap, 1u << 18);
  ix->stage_terms = ix->stage_rows * 64;
  FR_ALLOC(dalloc(&ix->d_rows, ix->stage_rows * ix->dim, D));
  FR_ALLOC(dalloc(&ix->d_off, ix->stage_rows + 1, D));
  FR_ALLOC(dalloc(&ix->d_tl, ix->stage_terms, D));
  FR_ALLOC(dalloc(&ix->d_ids, ix->stage_rows, D));
  FR_ALLOC(dalloc(&ix->d_slots, ix->stage_rows, D));
  FR_ALLOC(halloc(&ix->h_flag, 1, H));
  ix->ustage_rows = std::min<uint64_t>(cap, 1u << 14);
  // any one document fits: its distinct terms number at most the vocabulary
  ix->ustage_terms = std::max<uint64_t>(ix->ustage_rows * 64, ix->L ? ix->L : cfg->vocab);
  FR_ALLOC(dalloc(&ix->d_urows, ix->ustage_rows * ix->dim, D));
  FR_ALLOC(dalloc(&ix->d_uoff, ix->ustage_rows + 1, D));
  FR_ALLOC(dalloc(&ix->d_uterms, ix->ustage_terms, D));
  FR_ALLOC(dalloc(&ix->d_uids, ix->ustage_rows, D));
  FR_ALLOC(dalloc(&ix->d_uslots, ix->ustage_rows, D));
  FR_ALLOC(dalloc(&ix->d_dslots, ix->ustage_rows, D));
  FR_ALLOC(dalloc(&ix->d_doff, ix->ustage_rows + 1, D));
  FR_ALLOC(dalloc(&ix->d_dterms, ix->ustage_terms, D));
  FR_ALLOC(halloc(&ix->h_urows, ix->ustage_rows * ix->dim, H));
  FR_ALLOC(halloc(&ix->h_uoff, ix->ustage_rows + 1, H));
  FR_ALLOC(halloc(&ix->h_uterms, ix->ustage_terms, H));
  FR_ALLOC(halloc(&ix->h_uids, ix->ustage_rows, H));
  FR_ALLOC(halloc(&ix->h_uslots, ix->ustage_rows, H));
  FR_ALLOC(halloc(&ix->h_dslots, ix->ustage_rows, H));
  FR_ALLOC(halloc(&ix->h_doff, ix->ustage_rows + 1, H));
  FR_ALLOC(halloc(&ix->h_dterms, ix->ustage_terms, H));
  if (hipEventCreateWithFlags(&ix->ustage_free, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ix->upd_done, hipEventDisableTiming) != hipSuccess) {
    cleanup();
    return fail(FR_EDEVICE, "hipEventCreate failed");
  }

  const uint32_t nws = cfg->n_workspaces ? cfg->n_workspaces : 1;
  ix->ws.resize(nws);
  const uint32_t qm = ix->qmax, qpad = round_up(qm, kTile);
  const size_t n_in = 4 + (size_t)qm + (qm + 1) + (ix->cmax + 1) + ix->lmax + ix->batch_terms;
  for (auto& w : ix->ws) {
    const size_t bytes = layout_workspace(ix, w, nullptr, qm, ix->cmax, ix->lmax,
                                          cap / kGroup, ix->cand_cap, true);
    uint8_t* block = nullptr;
    FR_ALLOC(dalloc(&block, bytes, D));
    layout_workspace(ix, w, block, qm, ix->cmax, ix->lmax, cap / kGroup, ix->cand_cap, true);
    uint32_t* h_in = nullptr;
    FR_ALLOC(halloc(&h_in, n_in, H));
    layout_host_inputs(w, h_in);
    FR_ALLOC(halloc(&w.h_q, (size_t)qm * ix->dpad, H));
    FR_ALLOC(halloc(&w.h_ids, (size_t)qm * cfg->k_max, H));
    FR_ALLOC(halloc(&w.h_scores, (size_t)qm * cfg->k_max, H));
    FR_ALLOC(halloc(&w.h_count, qm, H));
    FR_ALLOC(halloc(&w.h_nmatch, qm, H));
    FR_ALLOC(halloc(&w.h_cnt, qm, H));
    FR_ALLOC(halloc(&w.h_selcnt, qm, H));
    FR_ALLOC(halloc(&w.h_desc_out, 4, H));
    bool ev_ok = hipEventCreate(&w.done) == hipSuccess;
    w.fin = w.done;
    // the call's start and the scan's bracket only time the device: no
    // system-scope fence (cache write-back and invalidation between the
    // kernels); the end event is also the host's completion event and keeps it
    for (int i = 0; i < Workspace::kRing && ev_ok; ++i)
      ev_ok = hipEventCreateWithFlags(&w.r0[i], hipEventDisableSystemFence) == hipSuccess &&
              hipEventCreateWithFlags(&w.r1[i], hipEventDisableSystemFence) == hipSuccess &&
              hipEventCreate(&w.r2[i]) == hipSuccess &&
              hipEventCreateWithFlags(&w.r3[i], hipEventDisableSystemFence) == hipSuccess;
    if (!ev_ok) {
      cleanup();
      return fail(FR_EDEVICE, "hipEventCreate failed");
    }
    std::memset(w.h_q, 0, (size_t)qm * ix->dpad * sizeof(float));
  }
  // fr_search_noalloc: the device's scratch (looked up once per device,
  // with the device current), its pinned input block and events
  {
    void* sp = nullptr;
    if (scratch_address(cfg->device, &sp) != hipSuccess) {
      cleanup();
      return fail(FR_EDEVICE, "hipGetSymbolAddress of the search scratch failed");
    }
    ix->scratch = (uint8_t*)sp;
  }
  FR_ALLOC(halloc(&ix->na_h_in, n_in, H));
  FR_ALLOC(halloc(&ix->na_h_count, qm, H));
  if (hipEventCreateWithFlags(&ix->na_copied, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ix->na_done, hipEventDisableTiming) != hipSuccess) {
    cleanup();
    return fail(FR_EDEVICE, "hipEventCreate failed");
  }
#undef FR_ALLOC
  // initial state: empty corpus, zero padding everywhere
  FR_HIP(launch_fill_u32((uint32_t*)ix->tiles, 0u, cap / kTile * tb / 4, ix->stream));
  if (ix->master) FR_HIP(launch_fill_u32((uint32_t*)ix->master, 0u, cap * ix->dpad, ix->stream));
  if (ix->xscale) FR_HIP(launch_fill_u32((uint32_t*)ix->xscale, 0x3F800000u, cap, ix->stream));
  FR_HIP(launch_fill_u32(ix->slot_ids, 0xFFFFFFFFu, cap, ix->stream));
  FR_HIP(launch_fill_u64(ix->live, 0ull, cap / 64, ix->stream));
  if (ix->L) FR_HIP(launch_fill_u32(ix->tcnt, 0u, cap, ix->stream));
  else FR_HIP(launch_fill_u64(ix->bits, 0ull, cap / kGroup * (uint64_t)cfg->vocab * kWords, ix->stream));
  FR_HIP(launch_fill_u32(ix->norm_max, 0u, 1, ix->stream));
  for (auto& w : ix->ws) {
    FR_HIP(launch_fill_u32((uint32_t*)w.qrow, 0u, (size_t)qm * ix->dpad, ix->stream));
    FR_HIP(launch_fill_u32((uint32_t*)w.qtiles, 0u, (size_t)qpad / kTile * tb / 4, ix->stream));
  }
  FR_HIP(hipStreamSynchronize(ix->stream));
  ix->slot_id.assign(cap, 0xFFFFFFFFu);
  ix->t_off.assign(cap, 0);
  ix->t_len.assign(cap, 0);
  *out = holder.release();
  return FR_OK;
}

fr_status fr_destroy(fr_index* ix) {
  if (!ix) return FR_OK;
  {
    std::lock_guard<std::mutex> lk(ix->mu);
    (void)hipSetDevice(ix->cfg.device);
    for (auto& w : ix->ws) {
      if (w.done) {
        (void)hipEventSynchronize(w.done);
        (void)hipEventDestroy(w.done);
      }
      drop_graph(w);
      for (int i = 0; i < Workspace::kRing; ++i) {
        if (w.r0[i]) (void)hipEventDestroy(w.r0[i]);
        if (w.r1[i]) (void)hipEventDestroy(w.r1[i]);
        if (w.r2[i]) (void)hipEventDestroy(w.r2[i]);
        if (w.r3[i]) (void)hipEventDestroy(w.r3[i]);
      }
    }
    if (ix->na_copied) {
      (void)hipEventSynchronize(ix->na_copied);
      (void)hipEventDestroy(ix->na_copied);
    }
    for (hipEvent_t e : {ix->na_done, ix->ustage_free, ix->upd_done})
      if (e) {
        (void)hipEventSynchronize(e);
        (void)hipEventDestroy(e);
      }
    if (ix->stream) {
      (void)hipStreamSynchronize(ix->stream);
      (void)hipStreamDestroy(ix->stream);
    }
    for (void* p : ix->dev_owned) (void)hipFree(p);
    for (void* p : ix->host_owned) (void)hipHostFree(p);
  }
  delete ix;
  return FR_OK;
}

fr_status fr_load_corpus(fr_index* ix, uint64_t n, const float* emb, const uint32_t* ids,
                         const uint64_t* term_off, const uint32_t* terms, uint32_t flags) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  FR_HIP(hipSetDevice(ix->cfg.device));
  const bool dev = flags & FR_DEVICE_PTRS;
  if (n > ix->cap || n > ix->cfg.capacity) return fail(FR_ECAPACITY, "n exceeds capacity");
  if (n && (!ids || !term_off)) return fail(FR_EINVAL, "ids / term_off missing");
  fr_status st = check_terms(ix, n, term_off, terms);
  if (st != FR_OK) return st;
  std::vector<uint32_t> hid(n);
  if (n) {
    if (dev) FR_HIP(hipMemcpy(hid.data(), ids, n * 4, hipMemcpyDeviceToHost));
    else std::memcpy(hid.data(), ids, n * 4);
  }
  std::unordered_map<uint32_t, uint32_t> m;
  m.reserve(n * 2 + 16);
  for (uint64_t i = 0; i < n; ++i) {
    if (hid[i] == 0xFFFFFFFFu) return fail(FR_EINVAL, "id 0xFFFFFFFF is reserved");
    if (!m.emplace(hid[i], (uint32_t)i).second)
      return fail(FR_EINVAL, "duplicate id " + std::to_string(hid[i]));
  }
  st = wait_all(ix);
  if (st != FR_OK) return st;
  st = check_rows(ix, emb, n, dev);
  if (st != FR_OK) return st;
  // reset the corpus
  const uint64_t used = std::max<uint64_t>(ix->hwm, 1);
  const uint64_t gused = (used + kGroup - 1) / kGroup;
  if (ix->L) FR_HIP(launch_fill_u32(ix->tcnt, 0u, gused * kGroup, ix->stream));
  else FR_HIP(launch_fill_u64(ix->bits, 0ull, gused * (uint64_t)ix->cfg.vocab * kWords, ix->stream));
  FR_HIP(launch_fill_u64(ix->live, 0ull, ix->cap / 64, ix->stream));
  FR_HIP(launch_fill_u32(ix->slot_ids, 0xFFFFFFFFu, ix->cap, ix->stream));
  FR_HIP(launch_fill_u32(ix->norm_max, 0u, 1, ix->stream));
  ix->id2slot.clear();
  ix->free_slots = decltype(ix->free_slots)();
  std::fill(ix->slot_id.begin(), ix->slot_id.end(), 0xFFFFFFFFu);
  ix->hwm = 0;
  ix->n_live = 0;
  st = write_docs(ix, n, emb, ids, term_off, terms, nullptr, 0, dev);
  if (st != FR_OK) {
    ix->failed = true;  // partially written corpus
    return st;
  }
  ix->id2slot.swap(m);
  for (uint64_t i = 0; i < n; ++i) ix->slot_id[i] = hid[i];
  // with headroom, so that inserts append without moving the arena (a
  // move copies every list while the index is locked); term lists need no
  // host copy (a delete clears nothing)
  if (!ix->L) {
    const uint64_t used = n ? term_off[n] - term_off[0] : 0;
    std::vector<uint32_t>().swap(ix->t_arena);
    ix->t_arena.reserve(used + used / 4 + (1u << 22));
    ix->t_arena.assign(n ? terms + term_off[0] : terms, n ? terms + term_off[n] : terms);
  }
  std::fill(ix->t_len.begin(), ix->t_len.end(), 0u);
  for (uint64_t i = 0; i < n && !ix->L; ++i) {
    ix->t_off[i] = term_off[i] - term_off[0];
    ix->t_len[i] = (uint32_t)(term_off[i + 1] - term_off[i]);
  }
  ix->t_garbage = 0;
  ix->hwm = n;
  ix->n_live = n;
  ix->epoch += 1;
  return FR_OK;
}

fr_status fr_update_docs(fr_index* ix, uint64_t n_del, const uint32_t* del_ids, uint64_t n_ins,
                         const uint32_t* ins_ids, const float* ins_emb,
                         const uint64_t* ins_term_off, const uint32_t* ins_terms,
                         uint64_t* out_epoch) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  FR_HIP(hipSetDevice(ix->cfg.device));
  if (n_del && !del_ids) return fail(FR_EINVAL, "del_ids missing");
  if (n_ins && (!ins_ids || !ins_term_off)) return fail(FR_EINVAL, "insert arrays missing");
  // validate everything first (all-or-nothing)
  std::unordered_set<uint32_t> dels;
  dels.reserve(n_del * 2 + 16);
  std::vector<uint32_t> del_slots(n_del);
  for (uint64_t i = 0; i < n_del; ++i) {
    auto it = ix->id2slot.find(del_ids[i]);
    if (it == ix->id2slot.end())
      return fail(FR_ENOTFOUND, "delete of unknown id " + std::to_string(del_ids[i]));
    if (!dels.insert(del_ids[i]).second)
      return fail(FR_ENOTFOUND, "id deleted twice in one call: " + std::to_string(del_ids[i]));
    del_slots[i] = it->second;
  }
  std::unordered_set<uint32_t> ins;
  ins.reserve(n_ins * 2 + 16);
  for (uint64_t i = 0; i < n_ins; ++i) {
    const uint32_t id = ins_ids[i];
    if (id == 0xFFFFFFFFu) return fail(FR_EINVAL, "id 0xFFFFFFFF is reserved");
    if (!ins.insert(id).second) return fail(FR_EDUPID, "id inserted twice: " + std::to_string(id));
    if (ix->id2slot.count(id) && !dels.count(id))
      return fail(FR_EDUPID, "insert of live id " + std::to_string(id));
  }
  if (ix->n_live - n_del + n_ins > ix->cfg.capacity)
    return fail(FR_ECAPACITY, "update exceeds capacity");
  fr_status st = check_terms(ix, n_ins, ins_term_off, ins_terms);
  if (st != FR_OK) return st;
  st = check_rows(ix, ins_emb, n_ins, false);
  if (st != FR_OK) return st;
  // the update runs on the index stream, behind every search in flight and
  // ahead of every search issued after this call; the host waits for no
  // search (only, past one staging chunk, for the previous chunk's copies)
  st = order_after_searches(ix);
  if (st != FR_OK) return st;
  std::vector<uint32_t> tmp;
  // deletes: live bit and slot id, then exactly the slot's own term bits
  for (uint64_t a0 = 0; a0 < n_del;) {
    st = stage_wait(ix);
    if (st != FR_OK) return st;
    uint64_t m = 0, nt = 0;
    ix->h_doff[0] = 0;
    while (a0 + m < n_del && m < ix->ustage_rows) {
      const uint32_t sl = del_slots[a0 + m];
      uint64_t len = ix->t_len[sl];
      const uint32_t* t = doc_terms(ix, ix->t_arena.data() + ix->t_off[sl], &len, tmp);
      if (nt + len > ix->ustage_terms) break;
      std::memcpy(ix->h_dterms + nt, t, len * 4);
      nt += len;
      ix->h_dslots[m++] = sl;
      ix->h_doff[m] = nt;
    }
    st = enqueue_deletes(ix, m, nt);
    if (st != FR_OK) {
      ix->failed = true;
      return st;
    }
    a0 += m;
  }
  for (uint64_t i = 0; i < n_del; ++i) {
    const uint32_t sl = del_slots[i];
    ix->id2slot.erase(del_ids[i]);
    ix->slot_id[sl] = 0xFFFFFFFFu;
    ix->free_slots.push(sl);
    ix->t_garbage += ix->t_len[sl];
    ix->t_len[sl] = 0;
  }
  ix->n_live -= n_del;
  // inserts: lowest free slots first
  std::vector<uint32_t> slots(n_ins);
  for (uint64_t i = 0; i < n_ins; ++i) {
    if (!ix->free_slots.empty()) {
      slots[i] = ix->free_slots.top();
      ix->free_slots.pop();
    } else {
      slots[i] = (uint32_t)ix->hwm++;
    }
  }
  for (uint64_t b0 = 0; b0 < n_ins;) {
    st = stage_wait(ix);
    if (st != FR_OK) return st;
    uint64_t m = 0, nt = 0;
    ix->h_uoff[0] = 0;
    while (b0 + m < n_ins && m < ix->ustage_rows) {
      const uint64_t i = b0 + m;
      uint64_t len = ins_term_off[i + 1] - ins_term_off[i];
      const uint32_t* t = doc_terms(ix, ins_terms + ins_term_off[i], &len, tmp);
      if (nt + len > ix->ustage_terms) break;
      std::memcpy(ix->h_uterms + nt, t, len * 4);
      std::memcpy(ix->h_urows + m * ix->dim, ins_emb + i * ix->dim, ix->dim * 4);
      nt += len;
      ix->h_uids[m] = ins_ids[i];
      ix->h_uslots[m++] = slots[i];
      ix->h_uoff[m] = nt;
    }
    st = enqueue_inserts(ix, m, nt);
    if (st != FR_OK) {
      ix->failed = true;
      return st;
    }
    b0 += m;
  }
  FR_HIP(hipEventRecord(ix->upd_done, ix->stream));
  ix->upd_pending = true;
  for (uint64_t i = 0; i < n_ins; ++i) {
    ix->id2slot[ins_ids[i]] = slots[i];
    ix->slot_id[slots[i]] = ins_ids[i];
    if (ix->L) continue;
    const uint64_t len = ins_term_off[i + 1] - ins_term_off[i];
    ix->t_off[slots[i]] = ix->t_arena.size();
    ix->t_len[slots[i]] = (uint32_t)len;
    ix->t_arena.insert(ix->t_arena.end(), ins_terms + ins_term_off[i],
                       ins_terms + ins_term_off[i] + len);
  }
  compact_terms(ix);
  ix->n_live += n_ins;
  ix->epoch += 1;
  if (out_epoch) *out_epoch = ix->epoch;
  return FR_OK;
}

fr_status fr_search(fr_index* ix, uint32_t n_q, const float* queries, const fr_cnf_batch* cnf,
                    const uint32_t* k, uint32_t* out_ids, float* out_scores, uint32_t* out_count,
                    uint64_t* out_nmatch, void* stream, uint32_t flags) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  FR_HIP(hipSetDevice(ix->cfg.device));
  const bool dev = flags & FR_DEVICE_PTRS;
  const bool async = stream || (flags & FR_ASYNC);
  if (async && !dev) return fail(FR_EINVAL, "an asynchronous search needs FR_DEVICE_PTRS");
  if ((flags & FR_GRAPH) && async && !stream)
    return fail(FR_EINVAL, "FR_GRAPH cannot capture the null stream");
  const bool pre = flags & FR_PRESELECT;
  if (pre && (!ix->qbits || !ix->quant_set))
    return fail(FR_EINVAL, "FR_PRESELECT needs an index created with quant_bits and an "
                           "encoding table (fr_set_quantizer)");
  if (pre && (flags & FR_GRAPH))
    return fail(FR_EUNSUPPORTED, "FR_PRESELECT searches are not captured (FR_GRAPH)");
  if (n_q > ix->qmax) return fail(FR_EINVAL, "n_q exceeds max_batch");
  uint32_t n_c = 0, n_l = 0;
  fr_status st = validate_cnf(ix, n_q, cnf, &n_c, &n_l);
  if (st != FR_OK) return st;
  if (n_q == 0) return FR_OK;
  if (!queries || !k || !out_ids || !out_scores || !out_count || !out_nmatch)
    return fail(FR_EINVAL, "null query or output pointer");
  for (uint32_t q = 0; q < n_q; ++q)
    if (k[q] > ix->cfg.k_max) return fail(FR_EINVAL, "k exceeds k_max");
  Workspace* w = acquire_ws(ix, flags & FR_NOWAIT, &st);
  if (!w) return st;
  hipStream_t s = async ? (hipStream_t)stream : ix->stream;
  st = order_after_update(ix, s);
  if (st != FR_OK) return st;
  // the call's timing slot; its start event goes before the input upload,
  // next to the previous call's end event (every event record between two
  // kernels costs the device a few microseconds)
  ring_slot(ix, *w);
  FR_HIP(hipEventRecord(w->e_start, s));
  // inputs
  w->h_desc[0] = n_q;
  w->h_desc[1] = n_q;
  w->h_desc[2] = 0;
  w->h_desc[3] = 0;
  std::memcpy(w->h_k, k, n_q * 4);
  st = stage_inputs(ix, *w, s, n_q, cnf, n_c, n_l);
  if (st != FR_OK) {
    ix->history.pop_back();   // nothing of the call ran
    w->n_calls -= 1;
    return st;
  }
  const size_t qbytes = (size_t)ix->dpad * 4;
  // device queries are read in place by the query tiling kernel
  const float* qsrc = dev ? queries : w->qrow;
  if (!dev) {
    for (uint32_t q = 0; q < n_q; ++q)
      std::memcpy(w->h_q + (size_t)q * ix->dpad, queries + (size_t)q * ix->dim, (size_t)ix->dim * 4);
    FR_HIP(hipMemcpyAsync(w->qrow, w->h_q, n_q * qbytes, hipMemcpyHostToDevice, s));
  }
  uint32_t* o_ids = dev ? out_ids : w->out_ids;
  float* o_scores = dev ? out_scores : w->out_scores;
  uint32_t* o_count = dev ? out_count : w->out_count;
  unsigned long long* o_nm = dev ? (unsigned long long*)out_nmatch : w->out_nmatch;
  const uint32_t n_groups = (uint32_t)((ix->hwm + kGroup - 1) / kGroup);
  const Choice ch = choose(ix, n_q, k, n_groups);
  uint64_t survivors = 0;   // pre-selection: sum over queries of min(quantK, live)
  if (pre) {
    uint32_t max_qk = 0;
    for (uint32_t q = 0; q < n_q; ++q) {
      const uint32_t qk = (uint32_t)std::min<uint64_t>((uint64_t)ix->qfactor * k[q], ix->scap);
      max_qk = std::max(max_qk, qk);
      survivors += std::min<uint64_t>(qk, ix->n_live);
    }
    st = enqueue_preselect(ix, *w, s, n_groups, max_qk, true, qsrc, o_ids, o_scores, o_count,
                           o_nm);
    if (st != FR_OK) return st;
  } else if (flags & FR_GRAPH) {
    // the whole device sequence as one graph, captured once per tiling,
    // corpus extent and output binding; kernels read the batch size from the
    // workspace descriptor, so any batch reuses the graph
    const uint64_t key[10] = {(uint64_t)ch.qb, (uint64_t)ch.nw, (uint64_t)ch.gpi, n_groups,
                             (uint64_t)(uintptr_t)o_ids, (uint64_t)(uintptr_t)o_scores,
                             (uint64_t)(uintptr_t)o_count, (uint64_t)(uintptr_t)o_nm,
                             (uint64_t)(uintptr_t)qsrc, (uint64_t)ch.strat};
    if (!w->gexec || std::memcmp(key, w->gkey, sizeof key) != 0) {
      drop_graph(*w);
      FR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      st = enqueue_search(ix, *w, s, ch, n_groups, false, qsrc, o_ids, o_scores, o_count, o_nm);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(s, &g);
      if (st != FR_OK) return st;
      FR_HIP(ce);
      w->graph = g;
      FR_HIP(hipGraphInstantiate(&w->gexec, g, nullptr, nullptr, 0));
      std::memcpy(w->gkey, key, sizeof key);
    }
    FR_HIP(hipEventRecord(w->e_scan0, s));
    FR_HIP(hipGraphLaunch(w->gexec, s));
    FR_HIP(hipEventRecord(w->e_scan1, s));
  } else {
    st = enqueue_search(ix, *w, s, ch, n_groups, true, qsrc, o_ids, o_scores, o_count, o_nm);
    if (st != FR_OK) return st;
  }
  const size_t kk = (size_t)n_q * ix->cfg.k_max;
  if (!dev) {
    FR_HIP(hipMemcpyAsync(w->h_ids, w->out_ids, kk * 4, hipMemcpyDeviceToHost, s));
    FR_HIP(hipMemcpyAsync(w->h_scores, w->out_scores, kk * 4, hipMemcpyDeviceToHost, s));
    FR_HIP(hipMemcpyAsync(w->h_count, w->out_count, n_q * 4, hipMemcpyDeviceToHost, s));
    FR_HIP(hipMemcpyAsync(w->h_nmatch, w->out_nmatch, n_q * 8, hipMemcpyDeviceToHost, s));
  }
  // the end of the call's device work: the timing ring's end event, which
  // the workspace's next user waits for
  FR_HIP(hipEventRecord(w->e_end, s));
  w->fin = w->e_end;
  w->in_flight = true;
  // algorithmic bytes / flops of this batch (for statistics)
  {
    std::vector<uint32_t> t(cnf->terms, cnf->terms + n_l);
    std::sort(t.begin(), t.end());
    w->last_terms = (uint64_t)(std::unique(t.begin(), t.end()) - t.begin());
    w->last_live = ix->n_live;
    w->last_preselect = pre;
    w->last_survivors = survivors;
    if (pre) {
      // one pass over the codes and predicate bits (the scan makes two),
      // plus the survivors' FP32 rows; "flops" counts the survivors' FP32
      // multiply-adds only (the code scores are integer work)
      w->last_alg_bytes = (double)ix->n_live * (ix->qbits / 8.0 + w->last_terms / 8.0) +
                          (double)ix->hwm / 8.0 + (double)survivors * ix->dpad * 4.0;
      w->last_alg_flops = 2.0 * ix->dim * (double)survivors;
    } else {
      const double per_doc =
          (double)ix->dpad * elem_bytes(ix->dt) + (ix->dt == kFP8 ? 4.0 : 0.0);
      w->last_alg_bytes = (double)ix->n_live * per_doc +
                          (double)ix->n_live * w->last_terms / 8.0 + (double)ix->hwm / 8.0 +
                          (double)n_q * ix->cfg.k_max * 8.0;
      w->last_alg_flops = 2.0 * ix->dim * n_q * (double)ix->n_live;
    }
  }
  w->last_nq = n_q;
  ix->last_ws = (size_t)(w - ix->ws.data());
  ix->have_last = true;
  if (async) return FR_OK;
  FR_HIP(hipEventSynchronize(w->fin));
  w->in_flight = false;
  bool failed_q = false;
  const uint32_t* cnts = w->h_count;
  if (dev) {
    FR_HIP(hipMemcpy(w->h_count, out_count, (size_t)n_q * 4, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out_ids, w->h_ids, kk * 4);
    std::memcpy(out_scores, w->h_scores, kk * 4);
    std::memcpy(out_count, w->h_count, n_q * 4);
    std::memcpy(out_nmatch, w->h_nmatch, n_q * 8);
    if (ix->n_live) {
      std::vector<uint64_t> nm(out_nmatch, out_nmatch + n_q);
      std::nth_element(nm.begin(), nm.begin() + n_q / 2, nm.end());
      ix->last_sel = sel_bucket((double)nm[n_q / 2] / (double)ix->n_live);
    }
  }
  for (uint32_t q = 0; q < n_q; ++q) failed_q |= cnts[q] == 0xFFFFFFFFu;
  if (failed_q)
    return fail(FR_EUNSUPPORTED,
                "a query had more tied candidates than the candidate buffer holds (raise cand_cap)");
  return FR_OK;
}

fr_status fr_search_noalloc(fr_index* ix, uint32_t n_q, const float* queries,
                            const fr_cnf_batch* cnf, const uint32_t* k, uint32_t* out_ids,
                            float* out_scores, uint32_t* out_count, uint64_t* out_nmatch,
                            void* stream, uint32_t flags) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  if (!(flags & FR_DEVICE_PTRS))
    return fail(FR_EINVAL, "fr_search_noalloc takes device queries and outputs (FR_DEVICE_PTRS)");
  if (flags & (FR_GRAPH | FR_NOWAIT))
    return fail(FR_EINVAL, "FR_GRAPH and FR_NOWAIT do not apply to fr_search_noalloc");
  FR_HIP(hipSetDevice(ix->cfg.device));
  const bool async = stream || (flags & FR_ASYNC);
  if (n_q > ix->qmax) return fail(FR_EINVAL, "n_q exceeds max_batch");
  uint32_t n_c = 0, n_l = 0;
  fr_status st = validate_cnf(ix, n_q, cnf, &n_c, &n_l);
  if (st != FR_OK) return st;
  if (n_q == 0) return FR_OK;
  if (!queries || !k || !out_ids || !out_scores || !out_count || !out_nmatch)
    return fail(FR_EINVAL, "null query or output pointer");
  for (uint32_t q = 0; q < n_q; ++q)
    if (k[q] > ix->cfg.k_max) return fail(FR_EINVAL, "k exceeds k_max");
  // this call's workspace, laid out in the device's scratch array
  const uint32_t n_groups = (uint32_t)((ix->hwm + kGroup - 1) / kGroup);
  Workspace w;
  const size_t need = layout_workspace(ix, w, nullptr, n_q, n_c, n_l, n_groups, ix->cand_cap, false);
  if (need > kScratchBytes)
    return fail(FR_EINVAL, "fr_search_noalloc: " + std::to_string(n_q) + " queries over " +
                               std::to_string(n_groups) + " groups of 1024 documents need " +
                               std::to_string(need >> 20) + " MiB of scratch, more than its " +
                               std::to_string(kScratchBytes >> 20) + " MiB (use fewer queries, or fr_search)");
  layout_workspace(ix, w, ix->scratch, n_q, n_c, n_l, n_groups, ix->cand_cap, false);
  // the pinned input block is reused: the previous call's copy must be done
  if (ix->na_pending) {
    FR_HIP(hipEventSynchronize(ix->na_copied));
    ix->na_pending = false;
  }
  layout_host_inputs(w, ix->na_h_in);
  hipStream_t s = async ? (hipStream_t)stream : ix->stream;
  st = order_after_update(ix, s);
  if (st != FR_OK) return st;
  w.h_desc[0] = n_q;
  w.h_desc[1] = n_q;
  w.h_desc[2] = 0;
  w.h_desc[3] = 0;
  std::memcpy(w.h_k, k, n_q * 4);
  st = stage_inputs(ix, w, s, n_q, cnf, n_c, n_l);
  if (st != FR_OK) return st;
  FR_HIP(hipEventRecord(ix->na_copied, s));
  ix->na_pending = true;
  const Choice ch = choose(ix, n_q, k, n_groups);
  st = enqueue_search(ix, w, s, ch, n_groups, false, queries, out_ids, out_scores, out_count,
                      (unsigned long long*)out_nmatch);
  if (st != FR_OK) return st;
  // (a search captured into the caller's graph is ordered by the caller)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  FR_HIP(hipStreamIsCapturing(s, &cs));
  if (cs == hipStreamCaptureStatusNone) {
    FR_HIP(hipEventRecord(ix->na_done, s));
    ix->na_inflight = true;
  }
  if (async) return FR_OK;
  FR_HIP(hipMemcpyAsync(ix->na_h_count, out_count, (size_t)n_q * 4, hipMemcpyDeviceToHost, s));
  FR_HIP(hipStreamSynchronize(s));
  for (uint32_t q = 0; q < n_q; ++q)
    if (ix->na_h_count[q] == 0xFFFFFFFFu)
      return fail(FR_EUNSUPPORTED,
                  "a query had more tied candidates than the candidate buffer holds (raise cand_cap)");
  return FR_OK;
}

fr_status fr_set_quantizer(fr_index* ix, const uint32_t* bin_off, const uint32_t* bin_dim,
                           const float* bin_sign) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  if (!ix->qbits) return fail(FR_EINVAL, "the index was created without quant_bits");
  if (!bin_off) return fail(FR_EINVAL, "bin_off missing");
  const uint32_t nb = ix->qbits;
  if (bin_off[0] != 0) return fail(FR_EINVAL, "bin_off[0] must be 0");
  for (uint32_t j = 0; j < nb; ++j)
    if (bin_off[j + 1] < bin_off[j]) return fail(FR_EINVAL, "bin_off must be non-decreasing");
  const uint64_t ne = bin_off[nb];
  if (ne > ix->bin_cap)
    return fail(FR_EINVAL, "more table entries (" + std::to_string(ne) + ") than bits x padded "
                           "dimension (" + std::to_string(ix->bin_cap) + ")");
  if (ne && (!bin_dim || !bin_sign)) return fail(FR_EINVAL, "bin_dim / bin_sign missing");
  for (uint64_t e = 0; e < ne; ++e) {
    if (bin_dim[e] >= ix->dim) return fail(FR_EINVAL, "bin_dim entry >= dim");
    if (bin_sign[e] != 1.0f && bin_sign[e] != -1.0f)
      return fail(FR_EINVAL, "bin_sign entries must be +1 or -1");
  }
  FR_HIP(hipSetDevice(ix->cfg.device));
  fr_status st = wait_all(ix);
  if (st != FR_OK) return st;
  FR_HIP(hipMemcpyAsync(ix->d_bin_off, bin_off, (nb + 1) * 4, hipMemcpyHostToDevice, ix->stream));
  if (ne) {
    FR_HIP(hipMemcpyAsync(ix->d_bin_dim, bin_dim, ne * 4, hipMemcpyHostToDevice, ix->stream));
    FR_HIP(hipMemcpyAsync(ix->d_bin_sign, bin_sign, ne * 4, hipMemcpyHostToDevice, ix->stream));
  }
  ix->quant_set = true;
  // the corpus already stored: every slot from its FP32 master row
  hipError_t e = encode_rows(ix, ix->master, ix->dpad, ix->hwm, nullptr, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(ix->stream);
  if (e != hipSuccess) {
    ix->failed = true;
    return fail(FR_EDEVICE, std::string("encoding the corpus failed: ") + hipGetErrorString(e));
  }
  return FR_OK;
}

fr_status fr_debug_codes(fr_index* ix, uint64_t slot0, uint64_t n, uint64_t* out) {
  if (!ix || (n && !out)) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (!ix->qbits) return fail(FR_EINVAL, "the index has no sign codes");
  if (slot0 + n > ix->cap) return fail(FR_EINVAL, "slot range beyond capacity");
  FR_HIP(hipSetDevice(ix->cfg.device));
  fr_status st = wait_all(ix);
  if (st != FR_OK) return st;
  const uint32_t W = ix->qbits / 64;
  // whole 64-slot chunks covering the range, then rows in slot order
  const uint64_t c0 = slot0 / 64, c1 = (slot0 + n + 63) / 64;
  std::vector<uint64_t> buf((c1 - c0) * W * 64);
  if (!buf.empty())
    FR_HIP(hipMemcpy(buf.data(), ix->codes + c0 * W * 64, buf.size() * 8, hipMemcpyDeviceToHost));
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t sl = slot0 + i;
    for (uint32_t w = 0; w < W; ++w)
      out[i * W + w] = buf[((sl / 64 - c0) * W + w) * 64 + sl % 64];
  }
  return FR_OK;
}

fr_status fr_stats(fr_index* ix, fr_search_stats* out) {
  if (!ix || !out) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (!ix->have_last) return fail(FR_EINVAL, "no search yet");
  Workspace& w = ix->ws[ix->last_ws];
  if (hipEventSynchronize(w.fin) != hipSuccess) return fail(FR_EDEVICE, "event");
  // per-query counters of that search, still in its workspace (read here
  // rather than copied back by every search)
  if (hipMemcpy(w.h_cnt, w.cnt, w.last_nq * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(w.h_selcnt, w.sel_cnt, w.last_nq * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(w.h_desc_out, w.desc, 16, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FR_EDEVICE, "hipMemcpy");
  fr_search_stats s{};
  s.n_queries = w.last_nq;
  uint64_t cands = 0;
  const uint32_t passes = w.h_desc_out[2] ? 2 : 1;
  double gathers = 0;
  for (uint32_t q = 0; q < w.last_nq; ++q) {
    if (w.last_preselect) {
      cands += std::min(w.h_cnt[q], ix->scap);   // survivors (their rows are in alg_bytes)
      continue;
    }
    cands += std::min(w.h_cnt[q], ix->cand_cap);
    if (ix->dt != kF32) gathers += (double)w.h_selcnt[q] * ix->dpad * 4.0;
  }
  s.n_passes = passes;
  s.candidates = cands;
  s.n_live = w.last_live;
  s.n_terms_batch = w.last_terms;
  s.alg_bytes = w.last_alg_bytes + gathers;
  s.alg_flops = w.last_alg_flops;
  float ms = 0;
  if (hipEventElapsedTime(&ms, w.e_scan0, w.e_scan1) == hipSuccess) s.ms_scan = ms;
  if (hipEventElapsedTime(&ms, w.e_scan0, w.e_end) == hipSuccess) s.ms_total = ms;
  if (hipEventElapsedTime(&ms, w.e_start, w.e_end) == hipSuccess) s.ms_call = ms;
  s.n_sparse = w.last_preselect ? 0u : w.h_desc_out[3];
  *out = s;
  return FR_OK;
}

fr_status fr_timings(fr_index* ix, uint32_t max, float* scan_ms, float* total_ms, uint32_t* n) {
  if (!ix || !n) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  const size_t h = ix->history.size();
  const size_t m = std::min<size_t>(max, h);
  for (size_t i = 0; i < m; ++i) {
    const auto& e = ix->history[h - m + i];
    Workspace& w = ix->ws[e.first];
    if (hipEventSynchronize(w.r2[e.second]) != hipSuccess) return fail(FR_EDEVICE, "event");
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, w.r0[e.second], w.r1[e.second]) != hipSuccess ||
        hipEventElapsedTime(&b, w.r0[e.second], w.r2[e.second]) != hipSuccess)
      return fail(FR_EDEVICE, "hipEventElapsedTime");
    if (scan_ms) scan_ms[i] = a;
    if (total_ms) total_ms[i] = b;
  }
  *n = (uint32_t)m;
  return FR_OK;
}

fr_status fr_info(fr_index* ix, uint64_t* n_live, uint64_t* epoch, uint64_t* n_slots) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (n_live) *n_live = ix->n_live;
  if (epoch) *epoch = ix->epoch;
  if (n_slots) *n_slots = ix->hwm;
  return FR_OK;
}

fr_status fr_debug_masks(fr_index* ix, const fr_cnf_batch* cnf, uint64_t* out_bits,
                         uint64_t n_words_per_query) {
  if (!ix || !cnf || !out_bits) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  FR_HIP(hipSetDevice(ix->cfg.device));
  const uint32_t n_q = cnf->n_queries;
  if (n_q > ix->qmax) return fail(FR_EINVAL, "n_q exceeds max_batch");
  uint32_t n_c = 0, n_l = 0;
  fr_status st = validate_cnf(ix, n_q, cnf, &n_c, &n_l);
  if (st != FR_OK) return st;
  const uint64_t need = (ix->hwm + 63) / 64;
  if (n_words_per_query < need) return fail(FR_EINVAL, "n_words_per_query < ceil(n_slots/64)");
  if (!n_q || !need) return FR_OK;
  st = wait_all(ix);
  if (st != FR_OK) return st;
  // the search's own mask pass (prep + k_mask_words) in workspace 0, whose
  // word-major mask buffer is then read back: these are the words the scan
  // consumes
  Workspace& w = ix->ws[0];
  w.h_desc[0] = n_q;
  w.h_desc[1] = n_q;
  w.h_desc[2] = 0;
  w.h_desc[3] = 0;
  std::memset(w.h_k, 0, (size_t)n_q * 4);
  st = stage_inputs(ix, w, ix->stream, n_q, cnf, n_c, n_l);
  if (st != FR_OK) return st;
  const uint32_t n_groups = (uint32_t)((ix->hwm + kGroup - 1) / kGroup);
  FR_HIP(launch_prep(prep_args(ix, w), ix->stream));
  FR_HIP(batch_bits(ix, w, n_groups, ix->stream));
  const MaskWordArgs ma = mask_args(ix, w, n_groups);
  FR_HIP(launch_mask_words(ma, ix->stream));
  FR_HIP(hipStreamSynchronize(ix->stream));
  const size_t ppad = ma.ppad;
  std::vector<uint64_t> tmp((size_t)n_groups * kWords * ppad);
  FR_HIP(hipMemcpy(tmp.data(), w.mw, tmp.size() * 8, hipMemcpyDeviceToHost));
  for (uint32_t q = 0; q < n_q; ++q)
    for (uint64_t i = 0; i < need; ++i) out_bits[q * n_words_per_query + i] = tmp[i * ppad + q];
  return FR_OK;
}

fr_status fr_debug_slots(fr_index* ix, uint32_t* out_ids, uint64_t n) {
  if (!ix || !out_ids) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  for (uint64_t i = 0; i < n; ++i) out_ids[i] = i < ix->slot_id.size() ? ix->slot_id[i] : 0xFFFFFFFFu;
  return FR_OK;
}

fr_status fr_debug_candidates(fr_index* ix, uint32_t n_q, uint32_t* out_ids, float* out_scores,
                              uint32_t* out_count) {
  if (!ix || !out_ids || !out_scores || !out_count) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (!ix->have_last) return fail(FR_EINVAL, "no search yet");
  Workspace& w = ix->ws[ix->last_ws];
  if (n_q > w.last_nq) return fail(FR_EINVAL, "n_q exceeds the last batch");
  FR_HIP(hipEventSynchronize(w.fin));
  const size_t R = ix->rmax;
  std::vector<unsigned long long> keys((size_t)n_q * R);
  std::vector<uint32_t> cnt(n_q);
  FR_HIP(hipMemcpy(keys.data(), w.sel_key, keys.size() * 8, hipMemcpyDeviceToHost));
  FR_HIP(hipMemcpy(cnt.data(), w.sel_cnt, n_q * 4, hipMemcpyDeviceToHost));
  for (uint32_t q = 0; q < n_q; ++q) {
    out_count[q] = cnt[q];
    for (size_t r = 0; r < R; ++r) {
      const bool ok = r < cnt[q];
      const unsigned long long key = keys[q * R + r];
      const uint32_t k32 = (uint32_t)(key >> 32);
      uint32_t u = (k32 & 0x80000000u) ? (k32 & 0x7FFFFFFFu) : ~k32;
      float f;
      std::memcpy(&f, &u, 4);
      out_ids[q * R + r] = ok ? 0xFFFFFFFFu - (uint32_t)key : 0xFFFFFFFFu;
      out_scores[q * R + r] = ok ? f : -INFINITY;
    }
  }
  return FR_OK;
}

fr_status fr_debug_rows(fr_index* ix, uint64_t slot0, uint64_t n, void* out_codes,
                        float* out_scales) {
  if (!ix || !out_codes) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->failed) return fail(FR_EDEVICE, "index failed earlier");
  if (slot0 + n > ix->cap) return fail(FR_EINVAL, "slot range outside capacity");
  if (!n) return FR_OK;
  FR_HIP(hipSetDevice(ix->cfg.device));
  fr_status st = wait_all(ix);
  if (st != FR_OK) return st;
  const int es = elem_bytes(ix->dt);
  const size_t tb = tile_bytes(ix->dt, ix->dpad);
  const uint64_t t0 = slot0 / kTile, t1 = (slot0 + n + kTile - 1) / kTile;
  std::vector<uint8_t> raw((t1 - t0) * tb);
  FR_HIP(hipMemcpy(raw.data(), ix->tiles + t0 * tb, raw.size(), hipMemcpyDeviceToHost));
  uint8_t* out = (uint8_t*)out_codes;
  const int hd = (int)ix->dpad / 2, pc = 16 / es;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t slot = slot0 + i;
    const uint8_t* tile = raw.data() + (slot / kTile - t0) * tb;
    const int r = (int)(slot % kTile);
    for (int e = 0; e < (int)ix->dpad; ++e) {
      const int h = e / hd, p = e % hd, j = p / pc, idx = p % pc;
      std::memcpy(out + (i * ix->dpad + e) * es, tile + (size_t)(j * 64 + h * 32 + r) * 16 + idx * es,
                  es);
    }
  }
  if (out_scales) {
    if (ix->xscale) FR_HIP(hipMemcpy(out_scales, ix->xscale + slot0, n * 4, hipMemcpyDeviceToHost));
    else for (uint64_t i = 0; i < n; ++i) out_scales[i] = 1.0f;
  }
  return FR_OK;
}

fr_status fr_set_tiling(fr_index* ix, uint32_t query_blocks, uint32_t waves,
                        uint32_t groups_per_item) {
  if (!ix) return fail(FR_EINVAL, "null index");
  std::lock_guard<std::mutex> lk(ix->mu);
  if (query_blocks || waves) {
    if (!scan_supported(ix->dt, ix->dpad, (int)query_blocks, (int)waves))
      return fail(FR_EUNSUPPORTED, "no scan kernel with that tiling");
    ix->qb = (int)query_blocks;
    ix->nw = (int)waves;
  } else {
    ix->qb = ix->nw = 0;
  }
  ix->gpi = (int)std::min<uint32_t>(groups_per_item, 64);
  return FR_OK;
}

fr_status fr_set_strategy(fr_index* ix, uint32_t strategy, int pinned) {
  if (!ix) return fail(FR_EINVAL, "null index");
  if (!strategy_ok(strategy)) return fail(FR_EINVAL, "unknown strategy bits");
  std::lock_guard<std::mutex> lk(ix->mu);
  ix->strat = strategy;
  ix->strat_pinned = pinned != 0;
  return FR_OK;
}

fr_status fr_autotune(fr_index* ix, uint32_t n_q, const float* queries, const fr_cnf_batch* cnf,
                      const uint32_t* k, uint32_t flags, uint32_t* out_query_blocks,
                      uint32_t* out_waves, uint32_t* out_groups, uint32_t* out_strategy) {
  if (!ix) return fail(FR_EINVAL, "null index");
  if (flags & FR_DEVICE_PTRS) return fail(FR_EINVAL, "autotune takes host pointers");
  if (!n_q || !k) return fail(FR_EINVAL, "autotune needs a non-empty batch");
  const size_t kk = (size_t)n_q * ix->cfg.k_max;
  std::vector<uint32_t> ids(kk), cnt(n_q);
  std::vector<float> sc(kk);
  std::vector<uint64_t> nm(n_q);
  const int saved_qb = ix->qb, saved_nw = ix->nw, saved_g = ix->gpi;
  const uint32_t saved_strat = ix->strat;
  const bool saved_pin = ix->strat_pinned;
  auto restore = [&]() {
    ix->qb = saved_qb;
    ix->nw = saved_nw;
    ix->gpi = saved_g;
    ix->strat = saved_strat;
    ix->strat_pinned = saved_pin;
  };
  // median device time of `reps` searches (after one unmeasured) with the
  // given tiling and strategy
  auto timed = [&](int qb, int nw, int g, uint32_t strat, int reps, float* ms) -> fr_status {
    ix->qb = qb;
    ix->nw = nw;
    ix->gpi = g;
    ix->strat = strat;
    ix->strat_pinned = true;
    std::vector<float> t;
    for (int rep = 0; rep <= reps; ++rep) {
      fr_status st = fr_search(ix, n_q, queries, cnf, k, ids.data(), sc.data(), cnt.data(),
                               nm.data(), nullptr, 0);
      if (st != FR_OK) return st;
      fr_search_stats s{};
      st = fr_stats(ix, &s);
      if (st != FR_OK) return st;
      if (rep) t.push_back(s.ms_call);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return FR_OK;
  };
  struct Trial {
    int qb, nw, g;
    uint32_t strat;
    float ms;
  };
  // Untimed searches for kTunePrewarmMs first: in the first tenths of a
  // second of searching after an idle spell the GPU clocks higher than it
  // settles to under sustained load, which would favour the trials that
  // happen to run first.
  {
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::milliseconds(kTunePrewarmMs);
    int n = 0;
    while (n < 2 || std::chrono::steady_clock::now() < t_end) {
      fr_status st = fr_search(ix, n_q, queries, cnf, k, ids.data(), sc.data(), cnt.data(),
                               nm.data(), nullptr, 0);
      if (st != FR_OK) return st;
      ++n;
    }
  }
  // Stage 1: every tiling with the default strategy, then the other
  // strategies with the three fastest tilings, 3 timed searches each.
  // Stage 2: the three fastest trials again with 9 timed searches each
  // (near-equal candidates are told apart by the longer median).
  std::vector<Trial> trials;
  for (int nw : {4, 8}) {
    for (int qb : {1, 2, 4}) {
      if (!scan_supported(ix->dt, ix->dpad, qb, nw)) continue;
      const uint32_t qt = 32u * qb * nw;
      if (qt > round_up(n_q, 128) && qt > 128) continue;
      for (int g : {0, 1, 2, 4, 8}) {
        Trial t{qb, nw, g, 0u, 0.f};
        fr_status st = timed(qb, nw, g, 0u, 3, &t.ms);
        if (st != FR_OK) {
          restore();
          return st;
        }
        trials.push_back(t);
      }
    }
  }
  auto by_ms = [](const Trial& x, const Trial& y) { return x.ms < y.ms; };
  std::sort(trials.begin(), trials.end(), by_ms);
  const size_t n_top = std::min<size_t>(3, trials.size());
  for (size_t i = 0; i < n_top; ++i) {
    for (uint32_t strat : {FR_STRAT_NO_SPECULATION, FR_STRAT_NO_REFRESH,
                           FR_STRAT_NO_SPECULATION | FR_STRAT_NO_REFRESH}) {
      Trial t = trials[i];
      t.strat = strat;
      fr_status st = timed(t.qb, t.nw, t.g, strat, 3, &t.ms);
      if (st != FR_OK) {
        restore();
        return st;
      }
      trials.push_back(t);
    }
  }
  std::sort(trials.begin(), trials.end(), by_ms);
  trials.resize(std::min<size_t>(3, trials.size()));
  for (Trial& t : trials) {
    fr_status st = timed(t.qb, t.nw, t.g, t.strat, 9, &t.ms);
    if (st != FR_OK) {
      restore();
      return st;
    }
  }
  std::sort(trials.begin(), trials.end(), by_ms);
  // Stage 3: sparse routing levels on the winner (3 searches each), the
  // fastest level again with 9 against the winner without routing.
  {
    Trial base = trials[0], lv_best = base;
    lv_best.ms = INFINITY;
    for (uint32_t lv = 1; lv <= kSparseMaxLevel; ++lv) {
      Trial t = base;
      t.strat = (base.strat & ~FR_STRAT_SPARSE_MASK) | FR_STRAT_SPARSE(lv);
      fr_status st = timed(t.qb, t.nw, t.g, t.strat, 3, &t.ms);
      if (st != FR_OK) {
        restore();
        return st;
      }
      if (t.ms < lv_best.ms) lv_best = t;
    }
    if (lv_best.ms < base.ms) {
      fr_status st = timed(lv_best.qb, lv_best.nw, lv_best.g, lv_best.strat, 9, &lv_best.ms);
      if (st != FR_OK) {
        restore();
        return st;
      }
      if (lv_best.ms < base.ms) trials[0] = lv_best;
    }
  }
  const float best = trials[0].ms;
  const int best_qb = trials[0].qb, best_nw = trials[0].nw, best_g = trials[0].g;
  const uint32_t best_s = trials[0].strat;
  restore();
  // the batch's buckets (its selectivity from the last search's counts)
  uint32_t kmax = 0;
  for (uint32_t q = 0; q < n_q; ++q) kmax = std::max(kmax, sel_size(ix, k[q]));
  std::vector<uint64_t> m(nm);
  std::nth_element(m.begin(), m.begin() + n_q / 2, m.end());
  const int sb = sel_bucket(ix->n_live ? (double)m[n_q / 2] / (double)ix->n_live : 0.0);
  {
    std::lock_guard<std::mutex> lk(ix->mu);
    ix->tuned[std::make_tuple(q_bucket(n_q), q_bucket(kmax), sb)] =
        fr_index::Tuned{best_qb, best_nw, best_g, best_s, best};
    ix->last_sel = sb;
  }
  if (out_query_blocks) *out_query_blocks = (uint32_t)best_qb;
  if (out_waves) *out_waves = (uint32_t)best_nw;
  if (out_groups) *out_groups = (uint32_t)best_g;
  if (out_strategy) *out_strategy = best_s;
  return FR_OK;
}

fr_status fr_tuning_choice(fr_index* ix, uint32_t n_q, const uint32_t* k,
                           uint32_t* out_query_blocks, uint32_t* out_waves,
                           uint32_t* out_groups, uint32_t* out_strategy, uint32_t* out_source) {
  if (!ix || (n_q && !k)) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  const uint32_t n_groups = (uint32_t)((ix->hwm + kGroup - 1) / kGroup);
  const Choice c = choose(ix, n_q, k, n_groups);
  if (out_query_blocks) *out_query_blocks = (uint32_t)c.qb;
  if (out_waves) *out_waves = (uint32_t)c.nw;
  if (out_groups) *out_groups = (uint32_t)c.gpi;
  if (out_strategy) *out_strategy = c.strat;
  if (out_source) *out_source = (uint32_t)c.source;
  return FR_OK;
}

fr_status fr_tuning_save(fr_index* ix, const char* path) {
  if (!ix || !path) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(FR_EINVAL, std::string("cannot write ") + path);
  for (const auto& e : ix->tuned)
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"dtype\": %d, \"dim\": %u, \"vocab\": %u, "
                 "\"q_bucket\": %d, \"k_bucket\": %d, \"sel_bucket\": %d, "
                 "\"query_blocks\": %d, \"waves\": %d, \"groups_per_item\": %d, "
                 "\"strategy\": %u, \"ms\": %.4f}\n",
                 ix->arch, ix->dt, ix->dim, ix->cfg.vocab, std::get<0>(e.first),
                 std::get<1>(e.first), std::get<2>(e.first), e.second.qb, e.second.nw,
                 e.second.gpi, e.second.strat, e.second.ms);
  const bool ok = std::fclose(f) == 0;
  if (!ok) return fail(FR_EINVAL, std::string("cannot write ") + path);
  return FR_OK;
}

fr_status fr_tuning_load(fr_index* ix, const char* path, uint32_t* out_loaded) {
  if (!ix || !path) return fail(FR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ix->mu);
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(FR_EINVAL, std::string("cannot read ") + path);
  char line[512];
  uint32_t n = 0;
  while (std::fgets(line, sizeof line, f)) {
    char arch[32] = {};
    int dt, qk, kk, sk, qb, nw, g;
    unsigned dim, vocab, strat;
    float ms;
    const int got = std::sscanf(
        line,
        " {\"arch\": \"%31[^\"]\", \"dtype\": %d, \"dim\": %u, \"vocab\": %u, "
        "\"q_bucket\": %d, \"k_bucket\": %d, \"sel_bucket\": %d, \"query_blocks\": %d, "
        "\"waves\": %d, \"groups_per_item\": %d, \"strategy\": %u, \"ms\": %f}",
        arch, &dt, &dim, &vocab, &qk, &kk, &sk, &qb, &nw, &g, &strat, &ms);
    if (got != 12) continue;                    // not an entry line
    if (std::strcmp(arch, ix->arch) || dt != ix->dt || dim != ix->dim || vocab != ix->cfg.vocab)
      continue;                                 // tuned for another index shape
    if (!scan_supported(ix->dt, ix->dpad, qb, nw) || g < 0 || g > 64 ||
        !strategy_ok(strat))
      continue;
    ix->tuned[std::make_tuple(qk, kk, sk)] = fr_index::Tuned{qb, nw, g, strat, ms};
    ++n;
  }
  std::fclose(f);
  if (out_loaded) *out_loaded = n;
  return FR_OK;
}

}  // extern "C"
