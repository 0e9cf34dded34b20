// Sign-code coarse pre-selection for gfx950 (Sec. 5.3, last paragraph; the
// appendix "Optimizing System on GPU", Quantization): an OP+ORP-like code of
// n_bits sign bits per document, a scan that scores every predicate match by
// the number of code bits it shares with the query (popcount of the
// complemented XOR), the quantK = factor * k best matches kept, and the FP32
// inner product of those survivors only (k_row_dots, fr_sparse.hip); the
// exact top-K of the survivors is then the search kernels' exact selection.
//
// The popcount score is integer and small (0..n_bits), so the cut is exact
// without any speculation: a histogram pass counts, per query, the matches
// at each score; the threshold score follows from the counts; a collect pass
// keeps everything above it and sets the ties at it aside, of which the
// lowest ids are taken.  Both passes are plain vector-ALU work (XNOR and
// popcount on 64-bit words, no matrix instructions): a wavefront holds the
// codes of 64 documents and walks a block of 32 queries, whose codes and
// per-slice mask words are wave-uniform (scalar registers).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {

// ------------------------------------------------------------- encoding
// One thread per (row, code word): bit b of word w is set iff the FP32 sum
// over bin 64w+b of sign * coordinate, added in table order from +0, is > 0.
// (sign is +-1, so each product is exact and only the additions round.)
__global__ __launch_bounds__(256) void k_sign_codes(SignArgs a) {
  const uint32_t W = a.n_bits / 64u;
  uint64_t n = a.n;
  if (a.n_dev) n = min(n, (uint64_t)*a.n_dev);
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= n * W) return;
  const uint64_t i = t / W;
  const uint32_t w = (uint32_t)(t % W);
  const float* row = a.rows + i * a.ld;
  unsigned long long word = 0ull;
  for (int b = 0; b < 64; ++b) {
    const uint32_t j = w * 64u + (uint32_t)b;
    float acc = 0.f;
    for (uint32_t e = a.bin_off[j]; e < a.bin_off[j + 1]; ++e)
      acc = acc + a.bin_sign[e] * row[a.bin_dim[e]];
    if (acc > 0.f) word |= 1ull << b;
  }
  if (a.corpus_layout) {
    const uint64_t slot = a.slots ? (uint64_t)a.slots[i] : a.slot_base + i;
    a.codes[((slot / 64u) * W + w) * 64u + slot % 64u] = word;
  } else {
    a.codes[i * W + w] = word;
  }
}
hipError_t launch_sign_codes(const SignArgs& a, hipStream_t s) {
  if (!a.n) return hipSuccess;
  FR_REQUIRE(a.rows);
  FR_REQUIRE(a.bin_off);
  FR_REQUIRE(a.bin_dim);
  FR_REQUIRE(a.bin_sign);
  FR_REQUIRE(a.codes);
  if (a.n_bits % 64u || a.n_bits < 64u || a.n_bits > 512u || a.ld < a.dim)
    return hipErrorInvalidValue;
  const uint64_t threads = a.n * (a.n_bits / 64u);
  hipLaunchKernelGGL(k_sign_codes, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------- code scans
// The block's query codes, copied once into LDS (a wavefront then reads
// each query's words as broadcasts instead of waiting on a scalar load per
// query).
template <int W>
__device__ __forceinline__ void load_query_codes(const QuantArgs& a, uint64_t* s_qc, uint32_t q0,
                                                 uint32_t nql) {
  for (uint32_t i = threadIdx.x; i < nql * (uint32_t)W; i += blockDim.x)
    s_qc[i] = a.qcode[(uint64_t)q0 * W + i];
}

// The wavefront's 64 documents (one per lane) against each query of the
// block: `visit(qi, score, matched)` for every query with at least one match
// among them.  Query codes (LDS) and mask words are uniform across the
// wavefront.
template <int W, typename Visit>
__device__ __forceinline__ void scan_slice(const QuantArgs& a, const uint64_t* s_qc, uint32_t sl,
                                           uint32_t q0, uint32_t nql, int lane, Visit&& visit) {
  uint64_t x[W];
#pragma unroll
  for (int w = 0; w < W; ++w) x[w] = a.codes[((uint64_t)sl * W + w) * 64u + lane];
  // lane l < nql holds the mask word of query q0 + l over this slice
  const uint64_t mk =
      lane < (int)nql ? a.mw[(uint64_t)sl * a.ppad + q0 + (uint32_t)lane] : 0ull;
  const uint32_t mlo = (uint32_t)mk, mhi = (uint32_t)(mk >> 32);
  for (uint32_t qi = 0; qi < nql; ++qi) {
    const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mhi, (int)qi) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)mlo, (int)qi);
    if (m == 0ull) continue;
    const uint64_t* y = s_qc + qi * W;
    uint32_t sc = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) sc += (uint32_t)__popcll(~(x[w] ^ y[w]));
    visit(qi, sc, ((m >> lane) & 1ull) != 0ull);
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_quant_hist(QuantArgs a) {
  __shared__ uint32_t s_hist[kQuantQB * 513];
  __shared__ uint64_t s_qc[kQuantQB * 8];
  const uint32_t nq = min(*a.n_dev, a.max_q);
  const uint32_t q0 = blockIdx.y * (uint32_t)kQuantQB;
  if (q0 >= nq) return;
  const uint32_t nql = min((uint32_t)kQuantQB, nq - q0);
  const uint32_t nb1 = a.n_bits + 1u;
  for (uint32_t i = threadIdx.x; i < kQuantQB * nb1; i += blockDim.x) s_hist[i] = 0u;
  load_query_codes<W>(a, s_qc, q0, nql);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t sl1 = min((blockIdx.x + 1u) * a.spb, a.n_slices);
  for (uint32_t sl = blockIdx.x * a.spb + (threadIdx.x >> 6); sl < sl1; sl += 4u)
    scan_slice<W>(a, s_qc, sl, q0, nql, lane, [&](uint32_t qi, uint32_t sc, bool hit) {
      if (hit) atomicAdd(&s_hist[qi * nb1 + sc], 1u);
    });
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nql * nb1; i += blockDim.x) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(a.hist + (uint64_t)(q0 + i / nb1) * nb1 + i % nb1, v);
  }
}

// Append this lane's value where `p` holds: one counter update per
// wavefront, positions in lane order; nothing is written at or past `cap`.
__device__ __forceinline__ void wave_append(bool p, uint32_t* counter, uint32_t* buf,
                                            uint32_t cap, uint32_t val, int lane) {
  const unsigned long long b = __ballot(p);
  if (b == 0ull) return;
  const int leader = __ffsll((long long)b) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(b));
  base = (uint32_t)__shfl((int)base, leader);
  if (p) {
    const uint32_t pos = base + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    if (pos < cap) buf[pos] = val;
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_quant_collect(QuantArgs a) {
  __shared__ uint64_t s_qc[kQuantQB * 8];
  const uint32_t nq = min(*a.n_dev, a.max_q);
  const uint32_t q0 = blockIdx.y * (uint32_t)kQuantQB;
  if (q0 >= nq) return;
  const uint32_t nql = min((uint32_t)kQuantQB, nq - q0);
  load_query_codes<W>(a, s_qc, q0, nql);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // the block's thresholds and flags, lane l holding query q0 + l, read
  // once: in the query loop they are wave-uniform register reads
  const uint32_t my_thr = lane < (int)nql ? a.thr[q0 + (uint32_t)lane] : 0u;
  const uint32_t my_flag = lane < (int)nql ? a.flag[q0 + (uint32_t)lane] : kQuantFail;
  const uint32_t sl1 = min((blockIdx.x + 1u) * a.spb, a.n_slices);
  for (uint32_t sl = blockIdx.x * a.spb + (threadIdx.x >> 6); sl < sl1; sl += 4u) {
    const uint32_t slot = sl * 64u + (uint32_t)lane;
    scan_slice<W>(a, s_qc, sl, q0, nql, lane, [&](uint32_t qi, uint32_t sc, bool hit) {
      const uint32_t q = q0 + qi;
      const uint32_t fl = (uint32_t)__builtin_amdgcn_readlane((int)my_flag, (int)qi);
      if (fl & kQuantFail) return;
      const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)my_thr, (int)qi);
      const bool all = (fl & kQuantAll) != 0u;
      wave_append(hit && (sc > t || (all && sc == t)), a.cnt + q,
                  a.surv + (uint64_t)q * a.scap, a.scap, slot, lane);
      wave_append(hit && !all && sc == t, a.ntie + q, a.ties + (uint64_t)q * a.tcap, a.tcap,
                  slot, lane);
    });
  }
}

template <int W>
hipError_t launch_quant_scan(const QuantArgs& a, bool collect, hipStream_t s) {
  const dim3 g((a.n_slices + a.spb - 1) / a.spb, (a.max_q + kQuantQB - 1) / kQuantQB);
  if (collect)
    hipLaunchKernelGGL(k_quant_collect<W>, g, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_quant_hist<W>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t quant_scan(const QuantArgs& a, bool collect, hipStream_t s) {
  FR_REQUIRE(a.codes);
  FR_REQUIRE(a.qcode);
  FR_REQUIRE(a.mw);
  FR_REQUIRE(a.n_dev);
  if (collect) {
    FR_REQUIRE(a.thr);
    FR_REQUIRE(a.flag);
    FR_REQUIRE(a.cnt);
    FR_REQUIRE(a.surv);
    FR_REQUIRE(a.ntie);
    FR_REQUIRE(a.ties);
  } else {
    FR_REQUIRE(a.hist);
  }
  if (!a.max_q || !a.n_slices) return hipSuccess;
  if (a.spb < 1 || a.ppad < a.max_q || a.ppad % 256u) return hipErrorInvalidValue;
  switch (a.n_bits) {
    case 64: return launch_quant_scan<1>(a, collect, s);
    case 128: return launch_quant_scan<2>(a, collect, s);
    case 256: return launch_quant_scan<4>(a, collect, s);
    case 512: return launch_quant_scan<8>(a, collect, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_quant_hist(const QuantArgs& a, hipStream_t s) { return quant_scan(a, false, s); }
hipError_t launch_quant_collect(const QuantArgs& a, hipStream_t s) { return quant_scan(a, true, s); }

// ------------------------------------------------------------ the cut
// One thread per query: quantK = min(factor * k, scap); the threshold t is
// the largest score with at least quantK matches at or above it; the
// matches above t are all kept and `need` more are taken from those at t.
// With fewer matches than quantK every match is kept.
__global__ __launch_bounds__(256) void k_quant_cut(QuantSelectArgs a) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nq = min(*a.n_dev, a.max_q);
  if (q >= nq) return;
  const uint32_t nb1 = a.n_bits + 1u;
  const uint32_t* h = a.hist + (uint64_t)q * nb1;
  const uint64_t qk = min((uint64_t)a.factor * a.k[q], (uint64_t)a.scap);
  uint32_t thr = a.n_bits + 1u, need = 0u, fl = 0u;   // quantK = 0: nothing survives
  if (qk) {
    uint64_t above = 0;
    int t = (int)a.n_bits;
    for (; t >= 0; --t) {
      if (above + h[t] >= qk) break;
      above += h[t];
    }
    if (t < 0) {
      thr = 0u;
      fl = kQuantAll;
    } else {
      thr = (uint32_t)t;
      need = (uint32_t)(qk - above);
      if (need == h[t]) fl = kQuantAll;
      else if (h[t] > a.tcap) fl = kQuantFail;
    }
  }
  a.thr[q] = thr;
  a.need[q] = need;
  a.flag[q] = fl;
  a.cnt[q] = 0u;
  a.ntie[q] = 0u;
  a.tau[q] = 0u;
  a.hinvw[q] = 0.f;
  a.tsafe[q] = 0u;
  a.ovf[q] = 0u;
}
hipError_t launch_quant_cut(const QuantSelectArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.k);
  FR_REQUIRE(a.hist);
  FR_REQUIRE(a.thr);
  FR_REQUIRE(a.need);
  FR_REQUIRE(a.flag);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.ntie);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.hinvw);
  FR_REQUIRE(a.tsafe);
  FR_REQUIRE(a.ovf);
  if (!a.max_q) return hipSuccess;
  hipLaunchKernelGGL(k_quant_cut, dim3((a.max_q + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------- the ties
// One block per query: the `need` smallest ids among the ties at the
// threshold (ids are unique) by an MSB-first radix select over the tie
// buffer, then those ties join the survivors.
__global__ __launch_bounds__(256) void k_quant_ties(QuantSelectArgs a) {
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_digit, s_rank;
  const uint32_t q = blockIdx.x;
  const uint32_t nq = min(*a.n_dev, a.max_q);
  if (q >= nq) return;
  const uint32_t fl = a.flag[q];
  if (fl & kQuantFail) {
    if (threadIdx.x == 0) a.cnt[q] = a.scap + 1u;   // the exact selection marks it failed
    return;
  }
  const uint32_t need = a.need[q];
  if ((fl & kQuantAll) || need == 0u) return;
  const uint32_t n = min(a.ntie[q], a.tcap);
  const uint32_t* tl = a.ties + (uint64_t)q * a.tcap;
  uint32_t prefix = 0u, pmask = 0u;
  if (threadIdx.x == 0) s_rank = need;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t id = a.slot_ids[tl[i]];
      if ((id & pmask) == prefix) atomicAdd(&s_hist[(id >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0, rank = s_rank, d = 0;
      for (; d < 255u; ++d) {
        if (acc + s_hist[d] >= rank) break;
        acc += s_hist[d];
      }
      s_digit = d;
      s_rank = rank - acc;
    }
    __syncthreads();
    prefix |= s_digit << shift;
    pmask |= 255u << shift;
  }
  // prefix is the need-th smallest id
  uint32_t* sv = a.surv + (uint64_t)q * a.scap;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t slot = tl[i];
    if (a.slot_ids[slot] <= prefix) {
      const uint32_t pos = atomicAdd(a.cnt + q, 1u);
      if (pos < a.scap) sv[pos] = slot;
    }
  }
}
hipError_t launch_quant_ties(const QuantSelectArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.flag);
  FR_REQUIRE(a.need);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.ntie);
  FR_REQUIRE(a.ties);
  FR_REQUIRE(a.surv);
  FR_REQUIRE(a.slot_ids);
  if (!a.max_q) return hipSuccess;
  hipLaunchKernelGGL(k_quant_ties, dim3(a.max_q), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fr
