// Term lists for large vocabularies (appendix "TBR": the paper stores each
// document's attribute values as a list padded to maxNumAttr, with offsets,
// and checks a clause by intersecting sorted lists).  Per-term document
// bitmaps cost vocab/8 bytes per document, which a vocabulary of hundreds of
// thousands of values cannot afford; lists cost 4 bytes per document term.
// A search does not intersect lists per (query, document) pair: it turns
// the lists, once per batch, into bitmaps of the batch's own distinct terms
// (at most kBatchTermsMax), in the layout of the per-term bitmaps, and the
// predicate masks are then built by the same word-parallel pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {

// One thread per document: its terms into column j of its slot's chunk.
__global__ __launch_bounds__(256) void k_list_write(ListWriteArgs a) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t slot = a.slots ? (uint64_t)a.slots[i] : a.slot_base + i;
  const uint64_t o0 = a.off[i], o1 = a.off[i + 1];
  const uint32_t cnt = (uint32_t)min(o1 - o0, (uint64_t)a.L);
  uint32_t* col = a.tlist + (slot / 64u) * (uint64_t)a.L * 64u + slot % 64u;
  for (uint32_t j = 0; j < cnt; ++j) col[(uint64_t)j * 64u] = a.terms[o0 + j];
  a.tcnt[slot] = cnt;
}
hipError_t launch_list_write(const ListWriteArgs& a, hipStream_t s) {
  if (!a.n) return hipSuccess;
  FR_REQUIRE(a.off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.tlist);
  FR_REQUIRE(a.tcnt);
  if (!a.L) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_list_write, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Blocks of 4 wavefronts; a wavefront owns one 64-document word (group g,
// word w) at a time, one document per lane.  Each lane looks its terms up in
// the batch dictionary (binary search in LDS) and ORs its bit into the
// wavefront's LDS row of n_dict words; the wavefront then writes all n_dict
// words of (g, w), zeros included, so the bitmaps need no clearing.
__global__ __launch_bounds__(256) void k_batch_bits(BatchBitsArgs a) {
  __shared__ uint32_t s_dict[kBatchTermsMax];
  __shared__ unsigned long long s_acc[4][kBatchTermsMax];
  const uint32_t nd = a.n_dict;
  for (uint32_t i = threadIdx.x; i < nd; i += blockDim.x) s_dict[i] = a.dict[i];
  const int lane = threadIdx.x & 63;
  const uint32_t wv = threadIdx.x >> 6;
  unsigned long long* acc = s_acc[wv];
  const uint32_t n_words = a.n_groups * (uint32_t)kWords;
  for (uint32_t base = blockIdx.x * 4u; base < n_words; base += gridDim.x * 4u) {
    const uint32_t wid = base + wv;
    for (uint32_t u = (uint32_t)lane; u < nd; u += 64u) acc[u] = 0ull;
    __syncthreads();
    if (wid < n_words) {
      const uint64_t slot = (uint64_t)wid * 64u + (uint64_t)lane;
      const uint32_t cnt = a.tcnt[slot];
      const uint32_t* col = a.tlist + (uint64_t)wid * a.L * 64u + (uint32_t)lane;
      for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t t = col[(uint64_t)j * 64u];
        uint32_t lo = 0, hi = nd;   // first dictionary entry >= t
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_dict[mid] < t) lo = mid + 1u;
          else hi = mid;
        }
        if (lo < nd && s_dict[lo] == t) atomicOr(&acc[lo], 1ull << lane);
      }
    }
    __syncthreads();
    if (wid < n_words) {
      const uint32_t g = wid / (uint32_t)kWords, w = wid % (uint32_t)kWords;
      uint64_t* out = a.bits + (uint64_t)g * nd * kWords + w;
      for (uint32_t u = (uint32_t)lane; u < nd; u += 64u) out[(uint64_t)u * kWords] = acc[u];
    }
    __syncthreads();
  }
}
hipError_t launch_batch_bits(const BatchBitsArgs& a, hipStream_t s) {
  FR_REQUIRE(a.tlist);
  FR_REQUIRE(a.tcnt);
  FR_REQUIRE(a.dict);
  FR_REQUIRE(a.bits);
  if (a.n_dict > kBatchTermsMax || !a.L) return hipErrorInvalidValue;
  if (!a.n_dict || !a.n_groups) return hipSuccess;
  const uint32_t n_words = a.n_groups * (uint32_t)kWords;
  hipLaunchKernelGGL(k_batch_bits, dim3(grid_for((n_words + 3) / 4, 1, 8192)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fr
