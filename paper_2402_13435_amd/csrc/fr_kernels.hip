// HIP kernels of exhaustive filtered top-K retrieval for gfx950 (MI355X).
//
// The hot path (Sec. 5.3 "System Implementation" and the appendix
// "Optimizing System on GPU") is one fused scan per query batch:
//   predicate masks (F-TBR, CNF over per-term document bitmaps)
//   -> inner products on the matrix cores (F-EBR)
//   -> mask + running per-query threshold -> candidate append,
// followed by an exact per-query selection and, for the reduced-precision
// forms, an FP32 rescoring of the selected candidates.
//
// Layouts (all device memory is reserved when the index is created):
//  * embeddings: tiles of 32 rows.  Each row's dpad elements are split into
//    two halves; the 32 rows x 2 halves map to the 64 lanes of a wavefront,
//    and each lane's half-row is cut into 16-byte chunks stored as
//    [chunk][lane][16 B].  A wavefront therefore reads one chunk of a tile as
//    one contiguous kilobyte, and the registers it holds are directly the A
//    operand of the 32x32 matrix instructions (the k index is permuted so
//    that each 32-lane half owns a contiguous half of the dimension; a dot
//    product does not depend on the order of its terms).  Queries use the
//    same layout and act as the B operand held in registers for the whole
//    scan.  This plays the role of the paper's mixed row/column "float4"
//    layout (appendix, "Storing Dense Matrix").
//  * term bitmaps: for each group of 1024 documents and each term, one
//    128-byte run of 16 words (bit d of word w = document 64w+d of the
//    group holds the term).  A clause over the group is the OR of its
//    literals' runs; the CNF is the AND of the clauses (appendix, "TBR").
//  * live bits and slot ids per document slot.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fr_internal.h"

namespace fr {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------ order keys
// Scores map to 32-bit keys whose unsigned order is the float order
// (-0 and +0 share a key).  A candidate's 64-bit key appends the complement
// of its id, so the unsigned order of keys is (score desc, id asc) when
// sorted descending.
__device__ __forceinline__ uint32_t fkey(float s) {
  uint32_t u = __float_as_uint(s);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
  if (k <= kKeyNegInf) return -INFINITY;
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ quantizers
// BF16: round to nearest, ties to even, of a finite FP32 value.
__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
// OCP E4M3FN (bias 7, 3 mantissa bits, subnormals, max 448, no inf):
// nearest code, ties to even, saturating; zero encodes as 0x00.
__device__ __forceinline__ uint8_t to_e4m3_rne(float y) {
  const uint32_t u = __float_as_uint(y);
  const uint32_t sign = (u >> 31) << 7;
  const float a = fabsf(y);
  uint32_t code;
  if (a >= 448.0f) {
    code = 0x7Eu;
  } else if (a < 0.015625f) {               // below 2^-6: subnormal step 2^-9
    code = (uint32_t)__builtin_rintf(a * 512.0f);  // 0..8 (8 == 2^-6, code 0x08)
  } else {
    int e = (int)((u >> 23) & 0xFFu) - 127;  // -6..8
    const uint32_t frac = u & 0x7FFFFFu;
    uint32_t m = frac >> 20;
    const uint32_t rem = frac & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (m & 1u))) ++m;
    if (m == 8u) { m = 0u; ++e; }
    code = ((uint32_t)(e + 7) << 3) | m;
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return code ? (uint8_t)(sign | code) : (uint8_t)0;
}

// ------------------------------------------------------- small utilities
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Every launcher refuses a null pointer the kernel would dereference, so a
// host-side wiring mistake becomes an error status instead of a GPU fault.
#define FR_REQUIRE(p) \
  do {                \
    if (!(p)) return hipErrorInvalidValue; \
  } while (0)

static inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 65535u * 4) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------- tile rows
// One wavefront per row: FP32 row -> tiled storage in the index dtype
// (+ FP8 row scale, optional FP32 master copy, row norm).
template <int DT>
__global__ __launch_bounds__(256) void k_tile_rows(TileRowsArgs a) {
  constexpr int ES = DT == kF32 ? 4 : DT == kBF16 ? 2 : 1;
  constexpr int PC = 16 / ES;  // elements per 16-byte chunk
  const int lane = threadIdx.x & 63;
  const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  uint64_t n = a.n;
  if (a.n_dev) n = min(n, (uint64_t)*a.n_dev);
  if (row >= n) return;
  const uint64_t slot = a.slots ? (uint64_t)a.slots[row] : a.slot_base + row;
  const int dpad = (int)a.dpad, dim = (int)a.dim, hd = dpad / 2;
  float x[4];
  float ss = 0.f, amax = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = lane + 64 * i;
    x[i] = (e < dim) ? a.rows[row * (uint64_t)dim + e] : 0.f;
    ss = fmaf(x[i], x[i], ss);
    amax = fmaxf(amax, fabsf(x[i]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ss += __shfl_xor(ss, off);
    amax = fmaxf(amax, __shfl_xor(amax, off));
  }
  if (lane == 0) {
    const float nrm = sqrtf(ss);
    if (a.norm) a.norm[row] = nrm;
    if (a.norm_max) atomicMax(a.norm_max, __float_as_uint(nrm));
  }
  float inv = 1.f;
  if constexpr (DT == kFP8) {
    inv = amax > 0.f ? 448.0f / amax : 1.0f;
    if (lane == 0 && a.scale) a.scale[slot] = amax > 0.f ? amax / 448.0f : 1.0f;
  }
  const uint64_t tb = (uint64_t)kTile * dpad * ES;
  uint8_t* tile = a.tiles + (slot / kTile) * tb;
  const int r = (int)(slot % kTile);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = lane + 64 * i;
    if (e >= dpad) break;
    if (a.master) a.master[slot * (uint64_t)dpad + e] = x[i];
    const int h = e / hd, p = e % hd, j = p / PC, idx = p % PC;
    uint8_t* dst = tile + ((size_t)(j * 64 + h * 32 + r) * 16) + idx * ES;
    if constexpr (DT == kF32) {
      *(float*)dst = x[i];
    } else if constexpr (DT == kBF16) {
      *(uint16_t*)dst = to_bf16_rne(x[i]);
    } else {
      *dst = to_e4m3_rne(x[i] * inv);
    }
  }
}

hipError_t launch_tile_rows(const TileRowsArgs& a, hipStream_t s) {
  if (!a.n) return hipSuccess;
  FR_REQUIRE(a.rows);
  FR_REQUIRE(a.tiles);
  if (a.dt == kFP8) FR_REQUIRE(a.scale);
  if (a.dpad % 64 || a.dpad > 256 || a.dim > a.dpad) return hipErrorInvalidValue;
  const dim3 g((unsigned)((a.n + 3) / 4)), b(256);
  switch (a.dt) {
    case kF32: hipLaunchKernelGGL(k_tile_rows<kF32>, g, b, 0, s, a); break;
    case kBF16: hipLaunchKernelGGL(k_tile_rows<kBF16>, g, b, 0, s, a); break;
    default: hipLaunchKernelGGL(k_tile_rows<kFP8>, g, b, 0, s, a); break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------- bitmaps, live
__global__ __launch_bounds__(256) void k_terms(TermArgs a) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t slot = a.slots ? (uint64_t)a.slots[i] : a.slot_base + i;
  const uint64_t g = slot / kGroup;
  const uint32_t w = (uint32_t)((slot % kGroup) / 64);
  const unsigned long long bit = 1ull << (slot % 64);
  unsigned long long* base = (unsigned long long*)a.bits + g * (uint64_t)a.vocab * kWords + w;
  for (uint64_t j = a.off[i]; j < a.off[i + 1]; ++j) {
    unsigned long long* p = base + (uint64_t)a.terms[j] * kWords;
    if (a.set) atomicOr(p, bit);
    else atomicAnd(p, ~bit);
  }
}
hipError_t launch_terms(const TermArgs& a, hipStream_t s) {
  if (!a.n) return hipSuccess;
  FR_REQUIRE(a.off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.bits);
  hipLaunchKernelGGL(k_terms, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_live(LiveArgs a) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t slot = a.slots ? (uint64_t)a.slots[i] : a.slot_base + i;
  const unsigned long long bit = 1ull << (slot % 64);
  unsigned long long* w = (unsigned long long*)a.live + slot / 64;
  if (a.set) {
    a.slot_ids[slot] = a.ids[i];
    atomicOr(w, bit);
  } else {
    a.slot_ids[slot] = 0xFFFFFFFFu;
    atomicAnd(w, ~bit);
  }
}
hipError_t launch_live(const LiveArgs& a, hipStream_t s) {
  if (!a.n) return hipSuccess;
  FR_REQUIRE(a.slot_ids);
  FR_REQUIRE(a.live);
  if (a.set) FR_REQUIRE(a.ids);
  hipLaunchKernelGGL(k_live, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// One thread per (slot, term): clear the slot's bit in the term's run.
__global__ __launch_bounds__(256) void k_clear_slot_terms(const uint32_t* slots, uint64_t n,
                                                          uint64_t* bits, uint32_t vocab) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n * vocab) return;
  const uint64_t slot = slots[i / vocab];
  const uint64_t t = i % vocab;
  const uint64_t g = slot / kGroup;
  const unsigned long long bit = 1ull << (slot % 64);
  unsigned long long* p =
      (unsigned long long*)bits + (g * vocab + t) * kWords + (slot % kGroup) / 64;
  if (*p & bit) atomicAnd(p, ~bit);
}
hipError_t launch_clear_slot_terms(const uint32_t* slots, uint64_t n, uint64_t* bits,
                                   uint32_t vocab, hipStream_t s) {
  const uint64_t total = n * vocab;
  if (!total) return hipSuccess;
  FR_REQUIRE(slots);
  FR_REQUIRE(bits);
  hipLaunchKernelGGL(k_clear_slot_terms, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     slots, n, bits, vocab);
  return hipGetLastError();
}

__global__ void k_check_finite(const float* x, uint64_t n, uint32_t* flag) {
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}
hipError_t launch_check_finite(const float* x, uint64_t n, uint32_t* flag, hipStream_t s) {
  if (!n) return hipSuccess;
  FR_REQUIRE(x);
  FR_REQUIRE(flag);
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------- CNF masks
// Mask word w of group g for query q: live AND over clauses of (OR over the
// clause's literals of the term's bitmap word).  No clause -> live; an empty
// clause -> 0.
__device__ __forceinline__ uint64_t cnf_word(const uint64_t* __restrict__ live,
                                             const uint64_t* __restrict__ bits, uint32_t vocab,
                                             uint64_t g, int w, uint32_t q,
                                             const uint32_t* __restrict__ co,
                                             const uint32_t* __restrict__ lo,
                                             const uint32_t* __restrict__ terms) {
  uint64_t m = live[g * kWords + w];
  const uint32_t c0 = co[q], c1 = co[q + 1];
  const uint64_t* gb = bits + g * (uint64_t)vocab * kWords + w;
  for (uint32_t c = c0; c < c1 && m; ++c) {
    uint64_t cw = 0;
    const uint32_t l0 = lo[c], l1 = lo[c + 1];
    for (uint32_t l = l0; l < l1; ++l) cw |= gb[(uint64_t)terms[l] * kWords];
    m &= cw;
  }
  return m;
}

__global__ __launch_bounds__(256) void k_masks(MaskArgs a, uint64_t total) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint32_t q = (uint32_t)(i / a.n_words);
  const uint64_t wi = i % a.n_words;
  a.out[i] = cnf_word(a.live, a.bits, a.vocab, wi / kWords, (int)(wi % kWords), q, a.clause_off,
                      a.literal_off, a.terms);
}
hipError_t launch_masks(const MaskArgs& a, uint64_t total, hipStream_t s) {
  if (!total) return hipSuccess;
  FR_REQUIRE(a.live);
  FR_REQUIRE(a.bits);
  FR_REQUIRE(a.clause_off);
  FR_REQUIRE(a.literal_off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.out);
  hipLaunchKernelGGL(k_masks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, total);
  return hipGetLastError();
}

// ------------------------------------------------------------- prep
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n_q = *a.n_dev;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) a.work[threadIdx.x] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.n_list = n_q;
    *a.n_list2 = 0u;
  }
  if (q >= n_q || q >= a.max_q) return;
  const uint32_t k = a.k[q];
  uint32_t kp = k;
  if (a.dt != kF32 && k) {
    kp = max(a.rescore_min, 4u * k);
    kp = min(kp, a.rescore_r);
    kp = max(kp, k);
  }
  a.kp[q] = kp;
  a.tau[q] = kp ? kKeyNegInf : kKeyPosInf;
  a.cnt[q] = 0u;
  a.smax[q] = 0u;
  a.nmatch[q] = 0ull;
  a.ovf[q] = 0u;
  a.qlist[q] = q;
  const float m = __uint_as_float(*a.norm_max);
  const float hi = a.qnorm[q] * m * 1.0001f;
  a.hlo[q] = 0.f;
  a.hinvw[q] = (hi > 0.f && isfinite(hi)) ? (float)kNBF / hi : 0.f;
  uint32_t* h = a.hist + (uint64_t)q * kHist;
  for (int i = 0; i < kHist; ++i) h[i] = 0u;
  // literal table
  const uint32_t c0 = a.clause_off[q], c1 = a.clause_off[q + 1];
  const uint32_t l0 = c0 < c1 ? a.literal_off[c0] : 0u, l1 = c0 < c1 ? a.literal_off[c1] : 0u;
  const uint32_t nl = l1 - l0;
  uint32_t starts = 0, n = 0, empty = 0;
  constexpr uint32_t L = kLits;
  uint32_t* lit = a.lit + (uint64_t)q * L;
  for (uint32_t c = c0; c < c1; ++c) {
    const uint32_t a0 = a.literal_off[c], a1 = a.literal_off[c + 1];
    if (a0 == a1) empty = 1u;
    for (uint32_t l = a0; l < a1; ++l) {
      if (n < L) {
        if (l == a0) starts |= 1u << n;
        lit[n] = a.terms[l];
      }
      ++n;
    }
  }
  for (uint32_t i = n; i < L; ++i) lit[i] = 0u;
  a.linfo[q] = (nl > L ? L : nl) | (starts << 8) | (empty << 24) | ((nl > L ? 1u : 0u) << 25) |
               ((c1 > c0 ? 1u : 0u) << 26);
}
hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.k);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.qnorm);
  FR_REQUIRE(a.norm_max);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.smax);
  FR_REQUIRE(a.hist);
  FR_REQUIRE(a.hlo);
  FR_REQUIRE(a.hinvw);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.n_list2);
  FR_REQUIRE(a.work);
  FR_REQUIRE(a.ovf);
  FR_REQUIRE(a.clause_off);
  FR_REQUIRE(a.literal_off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.lit);
  FR_REQUIRE(a.linfo);
  hipLaunchKernelGGL(k_prep, dim3(grid_for(a.max_q ? a.max_q : 1, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rerun(RerunArgs a) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) a.work[threadIdx.x] = 0u;
  const uint32_t n_q = *a.n_dev;
  if (q >= n_q || q >= a.max_q || !a.ovf[q]) return;
  a.ovf[q] = 0u;
  const uint32_t p = atomicAdd(a.n_list2, 1u);
  a.qlist2[p] = q;
  // Raise the threshold from the complete first-pass histogram: the scan's
  // own refreshes may have seen only part of it.  Same bucket rule (and
  // one-bucket margin) as the scan's refresh.
  uint32_t* h = a.hist + (uint64_t)q * kHist;
  {
    const uint32_t kp = a.kp[q];
    const float lo0 = a.hlo[q], iw0 = a.hinvw[q];
    uint32_t suffix = 0;
    int bstar = -1;
    for (int c = kNBC - 1; c >= 0 && bstar < 0; --c) {
      if (suffix + h[c] < kp) {
        suffix += h[c];
        continue;
      }
      for (int f = 15; f >= 0; --f) {
        suffix += h[kNBC + c * 16 + f];
        if (suffix >= kp) {
          bstar = c * 16 + f;
          break;
        }
      }
      if (bstar < 0) bstar = c * 16;   // coarse and fine counts disagree: stay safe
    }
    if (kp && bstar >= 2 && iw0 > 0.f) {
      const uint32_t nk = fkey(lo0 + (float)(bstar - 1) / iw0);
      if (nk > a.tau[q]) a.tau[q] = nk;
    }
  }
  const float lo = fmaxf(key2f(a.tau[q]), 0.f);
  const float hi = key2f(a.smax[q]);
  const float span = (hi - lo) * 1.0001f;
  a.hlo[q] = lo;
  a.hinvw[q] = (span > 0.f && isfinite(span)) ? (float)kNBF / span : 0.f;
  a.cnt[q] = 0u;
  a.smax[q] = 0u;
  for (int i = 0; i < kHist; ++i) h[i] = 0u;
}
hipError_t launch_rerun(const RerunArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.ovf);
  FR_REQUIRE(a.qlist2);
  FR_REQUIRE(a.n_list2);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.smax);
  FR_REQUIRE(a.hist);
  FR_REQUIRE(a.hlo);
  FR_REQUIRE(a.hinvw);
  FR_REQUIRE(a.work);
  hipLaunchKernelGGL(k_rerun, dim3(grid_for(a.max_q ? a.max_q : 1, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_zero_work(uint32_t* w) {
  if (threadIdx.x < kXcds) w[threadIdx.x] = 0u;
}
hipError_t launch_zero_work(uint32_t* work, hipStream_t s) {
  FR_REQUIRE(work);
  hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(64), 0, s, work);
  return hipGetLastError();
}

// ------------------------------------------------------------- the scan
// Matrix-core products of one tile (A: 32 documents, from the LDS ring)
// with QB blocks of 32 queries (B, in registers).  The k order inside a
// 16-byte chunk is the same for both operands, so any fixed pairing of
// chunks gives the dot products.  A chunks are read from LDS one at a time
// and used for every query block before the next is read.
template <int DT, int CH, int QB>
__device__ __forceinline__ void mma_tile(f32x16 (&acc)[QB], const uint8_t* slot,
                                         const uint4 (&bq)[QB][CH], int lane) {
  const uint4* p = (const uint4*)slot + lane;
  if constexpr (DT == kF32) {
    // 32x32x2 FP32: a chunk holds 4 consecutive k values per lane
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const uint4 x = p[j * 64];
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x.x), __uint_as_float(bq[b][j].x), acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x.y), __uint_as_float(bq[b][j].y), acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x.z), __uint_as_float(bq[b][j].z), acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x.w), __uint_as_float(bq[b][j].w), acc[b], 0, 0, 0);
      }
    }
  } else if constexpr (DT == kBF16) {
    // 32x32x16 BF16: one chunk = the 8 k values of one instruction
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const uint4 x = p[j * 64];
#pragma unroll
      for (int b = 0; b < QB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x),
                                                          __builtin_bit_cast(bf16x8, bq[b][j]),
                                                          acc[b], 0, 0, 0);
    }
  } else {
    // 32x32x64 FP8 (E4M3, format code 0 for both operands, no block scale):
    // two chunks = the 32 k values of one instruction
#pragma unroll
    for (int j = 0; j < CH; j += 2) {
      const uint4 x0 = p[j * 64], x1 = p[(j + 1) * 64];
      const i32x8 av = {(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                        (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        const i32x8 bv = {(int)bq[b][j].x, (int)bq[b][j].y, (int)bq[b][j].z, (int)bq[b][j].w,
                          (int)bq[b][j + 1].x, (int)bq[b][j + 1].y, (int)bq[b][j + 1].z,
                          (int)bq[b][j + 1].w};
        acc[b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[b], 0, 0, 0, 0, 0, 0);
      }
    }
  }
}

// Row (within the 32-row tile) of accumulator element v of a lane in half h.
__device__ __forceinline__ int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Ring of corpus tiles in LDS.  One wavefront of the workgroup (the loader)
// copies tiles straight from HBM into ring slots (global_load_lds, 16 bytes
// per lane: one instruction moves one kilobyte chunk, which is exactly the
// chunk-major tile layout); the compute wavefronts read them with plain LDS
// loads.  Keeping the tile loads on their own wavefront keeps them out of
// the compute wavefronts' memory counters, so candidate atomics and mask
// loads there never wait behind tile traffic.
template <int DT, int DPAD>
struct Ring {
  static constexpr int ES = DT == kF32 ? 4 : DT == kBF16 ? 2 : 1;
  static constexpr int CH = DPAD * ES / 32;   // 1 KB chunks per tile
  static constexpr int TB = CH * 1024;       // tile bytes
  static constexpr int L = CH + (DT == kFP8 ? 1 : 0);   // loads per tile
  // tiles in flight ahead of the one being scored: about 64 KB of ring,
  // at least 2, at most 8, and within the 6-bit memory counter
  static constexpr int PD0 = 65536 / TB - 1;
  static constexpr int PD1 = PD0 < 2 ? 2 : PD0 > 8 ? 8 : PD0;
  static constexpr int PD = (PD1 - 1) * L <= 63 ? PD1 : 63 / L + 1;
  static constexpr int NS = PD + 1;          // slots
};

__device__ __forceinline__ constexpr int vm_wait_code(int n) {
  // s_waitcnt with vmcnt(n) only (expcnt and lgkmcnt at their maximum)
  return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00;
}

// Workgroup barrier for LDS hand-offs: this wavefront's LDS accesses are
// complete before it arrives; memory accesses are not moved across it.
__device__ __forceinline__ void wg_barrier() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// Copy tile `tile` (and its FP8 row scales) into one ring slot.
template <int DT, int CH>
__device__ __forceinline__ void dma_tile(const uint8_t* __restrict__ tiles,
                                         const float* __restrict__ xscale, uint64_t tile,
                                         uint8_t* slot, float* sslot, int lane) {
  const uint4* src = (const uint4*)(tiles + tile * (uint64_t)(CH * 1024)) + lane;
#pragma unroll
  for (int j = 0; j < CH; ++j)
    __builtin_amdgcn_global_load_lds((const void*)(src + j * 64),
                                     (__attribute__((address_space(3))) void*)(slot + j * 1024),
                                     16, 0, 0);
  if constexpr (DT == kFP8) {
    if (lane < kTile)
      __builtin_amdgcn_global_load_lds((const void*)(xscale + tile * kTile + lane),
                                       (__attribute__((address_space(3))) void*)sslot, 4, 0, 0);
  }
}

// Wait until at most `younger` tiles' loads of this wavefront are in flight.
template <int L, int PD>
__device__ __forceinline__ void wait_tiles(uint32_t younger) {
  static_assert((PD - 1) * L <= 63, "memory counter range");
  switch (younger) {
    case 0: __builtin_amdgcn_s_waitcnt(vm_wait_code(0)); break;
    case 1: __builtin_amdgcn_s_waitcnt(vm_wait_code(1 * L)); break;
    case 2: if constexpr (PD > 2) { __builtin_amdgcn_s_waitcnt(vm_wait_code(2 * L)); break; }
    case 3: if constexpr (PD > 3) { __builtin_amdgcn_s_waitcnt(vm_wait_code(3 * L)); break; }
    case 4: if constexpr (PD > 4) { __builtin_amdgcn_s_waitcnt(vm_wait_code(4 * L)); break; }
    case 5: if constexpr (PD > 5) { __builtin_amdgcn_s_waitcnt(vm_wait_code(5 * L)); break; }
    case 6: if constexpr (PD > 6) { __builtin_amdgcn_s_waitcnt(vm_wait_code(6 * L)); break; }
    case 7: if constexpr (PD > 7) { __builtin_amdgcn_s_waitcnt(vm_wait_code(7 * L)); break; }
    default: __builtin_amdgcn_s_waitcnt(vm_wait_code(0)); break;
  }
}

// FP8 row scales of the lane's 16 accumulator rows from a ring slot
__device__ __forceinline__ void read_scales(float4 (&xs)[4], const float* sslot, int lane) {
  const float4* s = (const float4*)sslot + (lane >> 5);
#pragma unroll
  for (int g = 0; g < 4; ++g) xs[g] = s[2 * g];
}

// Literal table of one query (built by the prep kernel): up to kLits term
// ids and a packed info word (see PrepArgs).  A lane evaluates the CNF of a
// query over one 64-document word with all literal loads in flight at once.
__device__ __forceinline__ bool lit_slow(uint32_t info) { return (info >> 25) & 1u; }

struct MaskJob {
  uint64_t lw[kLits];
  uint64_t live;
};

__device__ __forceinline__ void mask_issue(MaskJob& j, const uint64_t* __restrict__ bits,
                                           const uint64_t* __restrict__ live, uint32_t vocab,
                                           uint64_t g, int w, uint32_t info,
                                           const uint32_t* term) {
  const uint32_t nlit = info & 31u;
  const uint64_t* gb = bits + g * (uint64_t)vocab * kWords + w;
  j.live = live[g * kWords + w];
#pragma unroll
  for (int i = 0; i < kLits; ++i) j.lw[i] = (i < (int)nlit) ? gb[(uint64_t)term[i] * kWords] : 0ull;
}

__device__ __forceinline__ uint64_t mask_combine(const MaskJob& j, uint32_t info) {
  if ((info >> 24) & 1u) return 0ull;           // an empty clause matches nothing
  if (!((info >> 26) & 1u)) return j.live;      // no clause: every live document
  const uint32_t nlit = info & 31u, starts = (info >> 8) & 0xFFFFu;
  uint64_t m = j.live, cw = 0ull;
#pragma unroll
  for (int i = 0; i < kLits; ++i) {
    if (i < (int)nlit) {
      if (i > 0 && ((starts >> i) & 1u)) {
        m &= cw;
        cw = 0ull;
      }
      cw |= j.lw[i];
    }
  }
  return m & cw;
}

// One pass of the fused scan.  A workgroup has NW compute wavefronts and
// two helpers, and takes work items (a chunk of 1024-document groups x a
// tile of NW*QB*32 queries) from its XCD's queue:
//   * the loader wavefront streams every tile of the item's groups into the
//     LDS ring, a few tiles ahead;
//   * compute wavefront w owns QB blocks of 32 queries (B operand in
//     registers).  Per tile it scores the tile on the matrix cores (unless
//     no query of it matches the tile), drops (doc, query) pairs that fail
//     the predicate mask or score below the query's threshold, and stages
//     the rest in LDS.  It also evaluates the next group's predicate masks
//     for its queries (loads issued a tile ahead);
//   * the keeper wavefront moves staged candidates to the global per-query
//     buffers and histograms every F tiles, and raises the thresholds from
//     the global histograms (a three-stage pipeline, one stage per F tiles,
//     so its loads have F tiles to arrive).  Compute wavefronts read the
//     thresholds from LDS at every tile.
// Compute wavefronts thus issue no global atomics and wait on no global
// loads in the tile loop, except when a staging buffer is full (then they
// append directly).  One workgroup barrier per tile hands over a ring slot
// and a staging half; every wavefront executes the same barrier sequence:
// two per item fetch, one after the item set-up, one per tile, one at the
// item end.
template <int DT, int DPAD, int QB, int NW>
__global__ __launch_bounds__((NW + 2) * 64) void k_scan(ScanArgs a) {
  using R = Ring<DT, DPAD>;
  constexpr int CH = R::CH;                 // 16-byte chunks per lane per tile
  constexpr int QT = NW * QB * 32;          // queries per work item
  constexpr int MS = kWords + 1;            // padded mask row (bank spread)
  constexpr int NJ = (QB + 1) / 2;          // mask-job queries per lane
  constexpr int F = 2;                      // tiles per keeper cycle
  constexpr int SCH = 256;                  // staged entries per wavefront and half
  constexpr int RJ = QT / 64;               // queries per keeper lane
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  static_assert(QT <= 256, "staged query index is one byte");
  static_assert((kGroup / kTile) % F == 0, "cycles tile a group");
  __shared__ __attribute__((aligned(16))) uint8_t s_ring[R::NS * R::TB];
  __shared__ __attribute__((aligned(16))) float s_rscale[DT == kFP8 ? R::NS * kTile : 4];
  __shared__ uint64_t s_mask[QT * MS];
  __shared__ uint32_t s_lit[QT * kLits];
  __shared__ uint32_t s_item;
  // per query of the item, index j = (wave * QB + b) * 32 + col
  __shared__ float s_thr[QT];
  __shared__ uint32_t s_qg[QT];             // batch query index, kNone if unused
  __shared__ uint32_t s_qkp[QT];            // selection size
  __shared__ float s_qlo[QT];
  __shared__ float s_qiw[QT];
  // staging: entries (score key << 32 | slot) and the query's j, by half
  __shared__ unsigned long long s_sk[2][NW][SCH];
  __shared__ uint8_t s_sq[2][NW][SCH];
  __shared__ uint32_t s_sn[2][NW];
  // keeper scratch
  __shared__ uint32_t s_hcnt[QT];
  __shared__ uint32_t s_hbase[QT];
  __shared__ uint32_t s_hmax[QT];
  __shared__ uint32_t s_dirty[QT / 32];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5,
            col = lane & 31;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t n_list = *a.n_list;
  const uint32_t n_qtiles = (n_list + QT - 1) / QT;
  const uint32_t n_chunks = (a.n_groups + a.gpi - 1) / a.gpi;
  const uint32_t my_chunks = n_chunks > xcd ? (n_chunks - xcd + kXcds - 1) / kXcds : 0u;
  const uint32_t my_items = my_chunks * n_qtiles;
  // the item's groups and tile count (identical in every wavefront)
  auto item_range = [&](uint32_t item, uint64_t& g0, uint64_t& g1) {
    const uint32_t chunk = (item / n_qtiles) * kXcds + xcd;
    g0 = (uint64_t)chunk * a.gpi;
    g1 = min(g0 + a.gpi, (uint64_t)a.n_groups);
  };
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  if (wave == NW) {
    // ---------------------------------------------------------- loader
    // Tile i of an item goes to slot i % NS; it is issued after tile
    // barrier i - PD, when every compute wavefront is done with the slot's
    // previous tile (i - NS = i - PD - 1).
    for (;;) {
      wg_barrier();
      const uint32_t item = s_item;
      wg_barrier();
      if (item >= my_items) break;
      uint64_t g0, g1;
      item_range(item, g0, g1);
      const uint32_t n_t = (uint32_t)(g1 - g0) * (kGroup / kTile);
      const uint64_t tile0 = g0 * (uint64_t)(kGroup / kTile);
      for (uint32_t i = 0; i < (uint32_t)R::PD && i < n_t; ++i)
        dma_tile<DT, CH>(a.tiles, a.xscale, tile0 + i, s_ring + (i % R::NS) * R::TB,
                         s_rscale + (i % R::NS) * kTile, lane);
      wg_barrier();                                   // set-up
      for (uint32_t i = 0; i < n_t; ++i) {
        const uint32_t left = n_t - 1 - i;
        wait_tiles<R::L, R::PD>(left < (uint32_t)(R::PD - 1) ? left : (uint32_t)(R::PD - 1));
        wg_barrier();                                 // tile i
        const uint32_t nx = i + R::PD;
        if (nx < n_t)
          dma_tile<DT, CH>(a.tiles, a.xscale, tile0 + nx, s_ring + (nx % R::NS) * R::TB,
                           s_rscale + (nx % R::NS) * kTile, lane);
      }
      wg_barrier();                                   // item end
    }
    return;
  }

  if (wave == NW + 1) {
    // ---------------------------------------------------------- keeper
    // Move the staged entries of one half to the global buffers: count per
    // query, reserve space with one atomic per query, scatter, add the
    // histogram buckets, raise the running maximum.
    auto flush_half = [&](int h) {
      uint32_t n[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t c = s_sn[h][w];
        n[w] = c < (uint32_t)SCH ? c : (uint32_t)SCH;
      }
#pragma unroll
      for (int w = 0; w < NW; ++w)
        for (uint32_t i = lane; i < n[w]; i += 64) atomicAdd(&s_hcnt[s_sq[h][w][i]], 1u);
      wave_sync();
      for (int j = lane; j < QT; j += 64) {
        const uint32_t c = s_hcnt[j];
        if (c) {
          s_hbase[j] = atomicAdd(a.cnt + s_qg[j], c);
          atomicOr(&s_dirty[j >> 5], 1u << (j & 31));
        }
        s_hcnt[j] = 0u;
      }
      wave_sync();
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        for (uint32_t i = lane; i < n[w]; i += 64) {
          const uint32_t j = s_sq[h][w][i];
          const unsigned long long key = s_sk[h][w][i];
          const uint32_t r = atomicAdd(&s_hcnt[j], 1u);
          const uint32_t pos = s_hbase[j] + r;
          const uint32_t qg = s_qg[j];
          if (pos < a.cap) a.cand_key[(uint64_t)qg * a.cap + pos] = key;
          const uint32_t k32 = (uint32_t)(key >> 32);
          const float fb = (key2f(k32) - s_qlo[j]) * s_qiw[j];
          const int bk = fb >= (float)(kNBF - 1) ? kNBF - 1 : (fb > 0.f ? (int)fb : 0);
          uint32_t* hq = a.hist + (uint64_t)qg * kHist;
          atomicAdd(hq + kNBC + bk, 1u);
          atomicAdd(hq + (bk >> 4), 1u);
          atomicMax(&s_hmax[j], k32);
        }
      }
      wave_sync();
      for (int j = lane; j < QT; j += 64) {
        const uint32_t m = s_hmax[j];
        if (m) atomicMax(a.smax + s_qg[j], m);
        s_hmax[j] = 0u;
        s_hcnt[j] = 0u;
      }
      if (lane < NW) s_sn[h][lane] = 0u;
      wave_sync();
    };

    // Threshold pipeline; lane owns queries j = lane + 64 r.  rstage: 0 idle,
    // 1 coarse counts in flight, 2 coarse counts used (fine counts to
    // issue), 3 fine counts in flight.  A cycle first uses the loads issued
    // one cycle earlier, then moves the staged entries, then issues the next
    // loads: loads are used only after a whole cycle, and never wait behind
    // the atomics issued in the same cycle.
    int rstage = 0;
    uint32_t rsel = 0;            // bit r: query j refreshed in this round
    uint32_t rc[RJ][16];          // coarse, then fine counts
    uint32_t rtau[RJ], rcut[RJ], rsuf[RJ];
    auto refresh_issue = [&]() {
      if (rstage == 0) {
        rsel = 0;
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const int j = lane + 64 * r;
          const uint32_t qg = s_qg[j];
          const bool d = (s_dirty[j >> 5] >> (j & 31)) & 1u;
          rtau[r] = qg != kNone ? ld_relaxed(a.tau + qg) : kKeyNegInf;
          if (qg != kNone && d) rsel |= 1u << r;
          const uint32_t* h = a.hist + (uint64_t)(qg != kNone ? qg : 0u) * kHist;
#pragma unroll
          for (int i = 0; i < kNBC; ++i) rc[r][i] = ((rsel >> r) & 1u) ? ld_relaxed(h + i) : 0u;
        }
        wave_sync();
        for (int i = lane; i < QT / 32; i += 64) s_dirty[i] = 0u;
        wave_sync();
        rstage = 1;
      } else if (rstage == 2) {
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const int j = lane + 64 * r;
          const uint32_t qg = s_qg[j];
          const bool me = rcut[r] != kNone;
          const uint32_t* h = a.hist + (uint64_t)(qg != kNone ? qg : 0u) * kHist + kNBC +
                              (me ? rcut[r] : 0u) * 16;
#pragma unroll
          for (int i = 0; i < 16; ++i) rc[r][i] = me ? ld_relaxed(h + i) : 0u;
        }
        rstage = 3;
      }
    };
    auto refresh_consume = [&]() {
      if (rstage == 1) {
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const int j = lane + 64 * r;
          const uint32_t qg = s_qg[j];
          if (qg != kNone) {
            const float t = key2f(rtau[r]);
            if (t > s_thr[j]) s_thr[j] = t;
          }
          const uint32_t k = qg != kNone ? s_qkp[j] : 0u;
          uint32_t suffix = 0, above = 0;
          int cs = -1;
#pragma unroll
          for (int i = kNBC - 1; i >= 0; --i) {
            const uint32_t ns = suffix + rc[r][i];
            if (cs < 0 && ns >= k) { cs = i; above = suffix; }
            suffix = ns;
          }
          const bool me = ((rsel >> r) & 1u) && k && cs >= 0;
          rcut[r] = me ? (uint32_t)cs : kNone;
          rsuf[r] = above;
        }
        rstage = 2;
      } else if (rstage == 3) {
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const int j = lane + 64 * r;
          if (rcut[r] == kNone) continue;
          const uint32_t qg = s_qg[j];
          const uint32_t k = s_qkp[j];
          uint32_t suffix = rsuf[r];
          int fs = -1;
#pragma unroll
          for (int i = 15; i >= 0; --i) {
            const uint32_t ns = suffix + rc[r][i];
            if (fs < 0 && ns >= k) fs = i;
            suffix = ns;
          }
          const int bstar = (int)rcut[r] * 16 + (fs < 0 ? 0 : fs);
          const float iw = s_qiw[j];
          if (bstar >= 2 && iw > 0.f) {
            const float t = s_qlo[j] + (float)(bstar - 1) / iw;
            if (t > s_thr[j]) s_thr[j] = t;
            // publish without waiting: other workgroups pick it up on their
            // next reload
            atomicMax(a.tau + qg, fkey(t));
          }
        }
        rstage = 0;
      }
    };
    // finish the round in flight (if any) at once
    auto refresh_drain = [&]() {
      while (rstage != 0) {
        refresh_consume();
        if (rstage == 2) refresh_issue();
      }
    };

    for (;;) {
      wg_barrier();
      const uint32_t item = s_item;
      wg_barrier();
      if (item >= my_items) break;
      uint64_t g0, g1;
      item_range(item, g0, g1);
      const uint32_t n_t = (uint32_t)(g1 - g0) * (kGroup / kTile);
      wg_barrier();                                   // set-up: s_qg, s_thr valid
      for (int i = lane; i < QT / 32; i += 64) s_dirty[i] = 0u;
      for (int j = lane; j < QT; j += 64) {
        s_hcnt[j] = 0u;
        s_hmax[j] = 0u;
      }
      rstage = 0;
      wave_sync();
      for (uint32_t i = 0; i < n_t; ++i) {
        wg_barrier();                                 // tile i
        if (i % F == 0 && i > 0) {
          // the previous cycle's half is complete.  While some query has no
          // threshold yet (the first cycles of an item), run a whole
          // refresh round at once: until then every match is a candidate.
          refresh_consume();
          flush_half((int)((i / F - 1) & 1u));
          bool cold = false;
          if (i <= 4 * F) {
#pragma unroll
            for (int r = 0; r < RJ; ++r) {
              const int j = lane + 64 * r;
              cold = cold || (s_qg[j] != kNone && s_thr[j] == -INFINITY);
            }
          }
          if (__ballot(cold)) {
            refresh_drain();
            refresh_issue();
            refresh_drain();
          } else {
            refresh_issue();
          }
        }
      }
      wg_barrier();                                   // item end
      refresh_consume();
      flush_half((int)((n_t / F - 1) & 1u));
      if (rstage == 2) refresh_issue();
      refresh_drain();
    }
    return;
  }

  // ------------------------------------------------------------ compute
  constexpr int NQW = 32 * QB;              // queries per wavefront
  // matrix-core B operand and per-query state, block b -> query column col
  uint4 bq[QB][CH];
  uint32_t qi[QB], kp[QB];
  float thr[QB], hlo[QB], hinv[QB], qs[QB];
  bool qv[QB];
  // mask jobs: this lane evaluates blocks b = half + 2j (j < NJ), column col;
  // their literal terms live in s_lit
  uint32_t jinfo[NJ], jq[NJ], jcnt[NJ];
  bool jv[NJ];
  if (wave == 0)
    for (int i = lane; i < 2 * NW; i += 64) s_sn[i / NW][i % NW] = 0u;

  auto my_pos = [&](uint32_t qt, int b) -> uint32_t {
    return qt * QT + (uint32_t)((wave * QB + b) * 32 + col);
  };
  auto my_j = [&](int b) -> int { return (wave * QB + b) * 32 + col; };
  auto smask = [&](int b, int c, int w) -> uint64_t& {
    return s_mask[((wave * QB + b) * 32 + c) * MS + w];
  };
  auto jterms = [&](int j) -> const uint32_t* {
    return s_lit + ((wave * QB + half + 2 * j) * 32 + col) * kLits;
  };

  // load the literal tables of this lane's mask-job queries for tile qt
  auto load_jobs = [&](uint32_t qt) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int b = half + 2 * j;
      const uint32_t pos = my_pos(qt, b);
      jv[j] = b < QB && pos < n_list;
      const uint32_t q = jv[j] ? a.qlist[pos] : 0u;
      jq[j] = q;
      jinfo[j] = jv[j] ? a.linfo[q] : 0u;
      jcnt[j] = 0u;
      if (b < QB) {
        const uint4* t = (const uint4*)(a.lit + (uint64_t)q * kLits);
        uint4* d = (uint4*)(s_lit + ((wave * QB + b) * 32 + col) * kLits);
#pragma unroll
        for (int i = 0; i < kLits / 4; ++i) d[i] = jv[j] ? t[i] : make_uint4(0, 0, 0, 0);
      }
    }
  };
  auto flush_counts = [&]() {
    if (!a.count_matches) return;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      if (jv[j] && jcnt[j]) atomicAdd(a.nmatch + jq[j], (unsigned long long)jcnt[j]);
  };
  // evaluate words w and w+1 of group g for the lane's jobs (loads of both
  // words in flight together)
  auto masks_words_sync = [&](uint64_t g, int w) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int b = half + 2 * j;
      if (b < QB) {
        uint64_t m0 = 0ull, m1 = 0ull;
        if (jv[j]) {
          if (lit_slow(jinfo[j])) {
            m0 = cnf_word(a.live, a.bits, a.vocab, g, w, jq[j], a.clause_off, a.literal_off, a.terms);
            m1 = cnf_word(a.live, a.bits, a.vocab, g, w + 1, jq[j], a.clause_off, a.literal_off,
                          a.terms);
          } else {
            MaskJob x0, x1;
            mask_issue(x0, a.bits, a.live, a.vocab, g, w, jinfo[j], jterms(j));
            mask_issue(x1, a.bits, a.live, a.vocab, g, w + 1, jinfo[j], jterms(j));
            m0 = mask_combine(x0, jinfo[j]);
            m1 = mask_combine(x1, jinfo[j]);
          }
        }
        jcnt[j] += (uint32_t)(__popcll(m0) + __popcll(m1));
        smask(b, col, w) = m0;
        smask(b, col, w + 1) = m1;
      }
    }
  };
  auto load_queries = [&](uint32_t qt) {
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      const uint32_t pos = my_pos(qt, b);
      qv[b] = pos < n_list;
      const uint32_t q = qv[b] ? a.qlist[pos] : 0u;
      qi[b] = q;
      kp[b] = qv[b] ? a.kp[q] : 0u;
      hlo[b] = qv[b] ? a.hlo[q] : 0.f;
      hinv[b] = qv[b] ? a.hinvw[q] : 0.f;
      qs[b] = (DT == kFP8 && qv[b]) ? a.qscale[q] : 1.f;
      thr[b] = (qv[b] && kp[b]) ? key2f(ld_relaxed(a.tau + q)) : INFINITY;
      if (half == 0) {
        const int j = my_j(b);
        s_qg[j] = (qv[b] && kp[b]) ? q : kNone;
        s_qkp[j] = kp[b];
        s_qlo[j] = hlo[b];
        s_qiw[j] = hinv[b];
        s_thr[j] = thr[b];
      }
      const uint4* p = (const uint4*)(a.qtiles + (uint64_t)(q / kTile) * (CH * 1024)) +
                       half * 32 + (q % kTile);
#pragma unroll
      for (int j = 0; j < CH; ++j) bq[b][j] = qv[b] ? p[j * 64] : make_uint4(0, 0, 0, 0);
    }
  };

  // ------------------------------------------------------------ items
  uint32_t cur_qt = 0xFFFFFFFFu;
  uint64_t pending_g = ~0ull;   // group whose masks are already in LDS
  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.work + xcd, 1u);
    wg_barrier();
    const uint32_t item = s_item;
    wg_barrier();
    if (item >= my_items) break;
    const uint32_t qt = item % n_qtiles;
    uint64_t g0, g1;
    item_range(item, g0, g1);

    if (qt != cur_qt) {
      if (cur_qt != 0xFFFFFFFFu) flush_counts();
      cur_qt = qt;
      load_queries(qt);
      load_jobs(qt);
      pending_g = ~0ull;
    }
    if (pending_g != g0) {
#pragma unroll 1
      for (int w = 0; w < kWords; w += 2) masks_words_sync(g0, w);
    }
    wg_barrier();                                     // set-up

    for (uint64_t g = g0; g < g1; ++g) {
      const bool has_next = g + 1 < g1;
      // tiles of this group that some query of this wavefront matches
      uint32_t act = 0;
#pragma unroll 1
      for (int w = 0; w < kWords; ++w) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < QB; ++b)
          if (kp[b]) o |= smask(b, col, w);
        if (__ballot((uint32_t)o != 0u)) act |= 1u << (2 * w);
        if (__ballot((uint32_t)(o >> 32) != 0u)) act |= 2u << (2 * w);
      }

      const uint64_t tile0 = g * (uint64_t)(kGroup / kTile);
      // next-group mask pipeline: word `mw_fly` has loads in flight
      int mw_next = has_next ? 0 : kWords;   // next word to issue
      int mw_fly = -1;                        // word in flight
      MaskJob mj[NJ];
      auto mask_issue_word = [&](int w) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (jv[j] && !lit_slow(jinfo[j]))
            mask_issue(mj[j], a.bits, a.live, a.vocab, g + 1, w, jinfo[j], jterms(j));
        mw_fly = w;
      };
      auto mask_finish_word = [&]() {
        const int w = mw_fly;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int b = half + 2 * j;
          if (b < QB) {
            uint64_t m = 0ull;
            if (jv[j])
              m = lit_slow(jinfo[j]) ? cnf_word(a.live, a.bits, a.vocab, g + 1, w, jq[j],
                                                a.clause_off, a.literal_off, a.terms)
                                     : mask_combine(mj[j], jinfo[j]);
            jcnt[j] += (uint32_t)__popcll(m);
            smask(b, col, w) = m;
          }
        }
        mw_fly = -1;
      };

      // one step per tile of the group: wait for the tile's ring slot, then
      // (if a query of this wavefront matches the tile) score it
      const uint32_t ti0 = (uint32_t)(g - g0) * (kGroup / kTile);   // item-relative tile
      auto body = [&](int t) {
        const uint32_t ti = ti0 + (uint32_t)t;
        const uint32_t rs = ti % (uint32_t)R::NS;
        const int h = (int)((ti / F) & 1u);
        wg_barrier();
        // words whose current-group tiles are all behind us can be replaced
        if (mw_fly >= 0 && 2 * mw_fly + 1 < t) mask_finish_word();
        if (mw_fly < 0 && mw_next < kWords && mw_next <= (t >> 1) + 1) mask_issue_word(mw_next++);
        if (!((act >> t) & 1u)) return;
#pragma unroll
        for (int b = 0; b < QB; ++b) thr[b] = s_thr[my_j(b)];
        f32x16 accs[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) accs[b][v] = 0.f;
        mma_tile<DT, CH, QB>(accs, s_ring + rs * R::TB, bq, lane);
        float4 xs[4];
        if constexpr (DT == kFP8) read_scales(xs, s_rscale + rs * kTile, lane);
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          f32x16& acc = accs[b];
          const uint32_t m32 = (uint32_t)(smask(b, col, t >> 1) >> ((t & 1) * 32));
          if constexpr (DT == kFP8) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float4 x4 = xs[v >> 2];
              const float sc = (v & 3) == 0 ? x4.x : (v & 3) == 1 ? x4.y : (v & 3) == 2 ? x4.z : x4.w;
              acc[v] = (acc[v] * qs[b]) * sc;
            }
          }
          const f32x16& s = acc;
          float mx = s[0];
#pragma unroll
          for (int v = 1; v < 16; ++v) mx = fmaxf(mx, s[v]);
          const bool cand = (m32 != 0u) && (mx >= thr[b]);
          if (__ballot(cand)) {
            uint32_t pm = 0;
            if (cand) {
#pragma unroll
              for (int v = 0; v < 16; ++v)
                if (((m32 >> acc_row(v, half)) & 1u) && s[v] >= thr[b]) pm |= 1u << v;
            }
            if (pm) {
              const uint32_t p0 = atomicAdd(&s_sn[h][wave], (uint32_t)__popc(pm));
              const uint32_t q = qi[b];
              const int jj = my_j(b);
              uint32_t r = 0;
#pragma unroll
              for (int v = 0; v < 16; ++v) {
                if ((pm >> v) & 1u) {
                  const uint64_t slot = (tile0 + t) * kTile + acc_row(v, half);
                  const uint32_t k32 = fkey(s[v]);
                  // the id (for the tie order) is looked up by the selection
                  const unsigned long long key =
                      ((unsigned long long)k32 << 32) | (unsigned long long)slot;
                  const uint32_t idx = p0 + r++;
                  if (idx < (uint32_t)SCH) {
                    s_sk[h][wave][idx] = key;
                    s_sq[h][wave][idx] = (uint8_t)jj;
                  } else {
                    // staging full: append directly
                    const uint32_t pos = atomicAdd(a.cnt + q, 1u);
                    if (pos < a.cap) a.cand_key[(uint64_t)q * a.cap + pos] = key;
                    const float fb = (s[v] - hlo[b]) * hinv[b];
                    const int bk = fb >= (float)(kNBF - 1) ? kNBF - 1 : (fb > 0.f ? (int)fb : 0);
                    uint32_t* hq = a.hist + (uint64_t)q * kHist;
                    atomicAdd(hq + kNBC + bk, 1u);
                    atomicAdd(hq + (bk >> 4), 1u);
                    atomicMax(a.smax + q, k32);
                    atomicOr(&s_dirty[jj >> 5], 1u << (jj & 31));
                  }
                }
              }
            }
          }
        }
      };

#pragma unroll 1
      for (int t = 0; t < kGroup / kTile; ++t) body(t);
      // finish the next group's masks
      if (mw_fly >= 0) mask_finish_word();
      while (mw_next < kWords) {
        mask_issue_word(mw_next++);
        mask_finish_word();
      }
      pending_g = has_next ? g + 1 : ~0ull;
    }
    wg_barrier();                                     // item end
  }
  if (cur_qt != 0xFFFFFFFFu) flush_counts();
}

// (dtype, padded dim, query blocks per wavefront, wavefronts per workgroup)
#define FR_SCAN_CASES(X) \
  X(kF32, 64, 1, 4) X(kF32, 128, 1, 4) X(kF32, 192, 1, 4) X(kF32, 256, 1, 4) \
  X(kBF16, 64, 2, 4) \
  X(kBF16, 64, 1, 4) X(kBF16, 128, 1, 4) X(kBF16, 192, 1, 4) X(kBF16, 256, 1, 4) \
  X(kFP8, 64, 1, 4) X(kFP8, 64, 2, 4) X(kFP8, 128, 1, 4) X(kFP8, 128, 2, 4) \
  X(kFP8, 192, 1, 4) X(kFP8, 256, 1, 4)

bool scan_supported(int dt, int dpad, int qb, int nw) {
#define FR_SUP(D, P, Q, W) if (dt == D && dpad == P && qb == Q && nw == W) return true;
  FR_SCAN_CASES(FR_SUP)
#undef FR_SUP
  return false;
}

hipError_t launch_scan(const ScanArgs& a, int dt, int dpad, int qb, int nw, int n_wg,
                       hipStream_t s) {
  FR_REQUIRE(a.tiles);
  FR_REQUIRE(a.live);
  FR_REQUIRE(a.bits);
  FR_REQUIRE(a.qtiles);
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.smax);
  FR_REQUIRE(a.hist);
  FR_REQUIRE(a.hlo);
  FR_REQUIRE(a.hinvw);
  FR_REQUIRE(a.cand_key);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.work);
  FR_REQUIRE(a.clause_off);
  FR_REQUIRE(a.literal_off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.lit);
  FR_REQUIRE(a.linfo);
  if (dt == kFP8) {
    FR_REQUIRE(a.xscale);
    FR_REQUIRE(a.qscale);
  }
  if (a.gpi < 1 || n_wg < 1) return hipErrorInvalidValue;
#define FR_LAUNCH(D, P, Q, W)                                                          \
  if (dt == D && dpad == P && qb == Q && nw == W) {                                    \
    hipLaunchKernelGGL((k_scan<D, P, Q, W>), dim3(n_wg), dim3((W + 2) * 64), 0, s, a); \
    return hipGetLastError();                                                          \
  }
  FR_SCAN_CASES(FR_LAUNCH)
#undef FR_LAUNCH
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ selection
__device__ void bitonic_desc(unsigned long long* key, uint32_t* val, int n) {
  // n is a power of two; sorts key[0..n) descending, carrying val if given.
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long x = key[i], y = key[ixj];
          const bool desc = (i & k) == 0;
          if (desc ? (x < y) : (x > y)) {
            key[i] = y;
            key[ixj] = x;
            if (val) {
              const uint32_t t = val[i];
              val[i] = val[ixj];
              val[ixj] = t;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Exact top-kp of one query's candidates (those at or above the final
// threshold), sorted by key descending = (score desc, id asc).
__global__ __launch_bounds__(256) void k_select(SelectArgs a) {
  __shared__ unsigned long long s_key[kSelCap];
  __shared__ uint32_t s_slot[kSelCap];
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_n, s_digit, s_rank;
  const uint32_t pos = blockIdx.x;
  if (pos >= *a.n_list) return;
  const uint32_t q = a.qlist[pos];
  const uint32_t kp = a.kp[q];
  const uint32_t c = a.cnt[q];
  if (c > a.cap) {
    // Candidates were dropped: leave the query for a second pass, or, if
    // this was it, mark it failed (count 0xFFFFFFFF, no ids).
    if (threadIdx.x == 0) {
      a.ovf[q] = 1u;
      a.sel_cnt[q] = 0u;
    }
    if (a.write_out && a.final_pass) {
      for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
        a.out_ids[(uint64_t)q * a.k_max + r] = 0xFFFFFFFFu;
        a.out_scores[(uint64_t)q * a.k_max + r] = -INFINITY;
      }
      if (threadIdx.x == 0) {
        a.out_count[q] = 0xFFFFFFFFu;
        a.out_nmatch[q] = a.nmatch[q];
      }
    }
    return;
  }
  const uint32_t tau = a.tau[q];
  const unsigned long long* ck = a.cand_key + (uint64_t)q * a.cap;
  // a candidate is stored as (score key, slot); its sort key is (score key,
  // complement of the slot's id)
  auto sort_key = [&](unsigned long long raw) -> unsigned long long {
    const uint32_t id = a.slot_ids[(uint32_t)raw];
    return (raw & 0xFFFFFFFF00000000ull) | (unsigned long long)(0xFFFFFFFFu - id);
  };
  if (threadIdx.x == 0) s_n = 0u;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
    const unsigned long long raw = ck[i];
    if ((uint32_t)(raw >> 32) >= tau) {
      const uint32_t p = atomicAdd(&s_n, 1u);
      if (p < kSelCap) {
        s_key[p] = sort_key(raw);
        s_slot[p] = (uint32_t)raw;
      }
    }
  }
  __syncthreads();
  uint32_t m = s_n;
  if (m > kSelCap) {
    // MSB-first radix select of the kp-th largest key (keys are unique).
    unsigned long long prefix = 0ull, pmask = 0ull;
    if (threadIdx.x == 0) s_rank = kp;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0u;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
        const unsigned long long raw = ck[i];
        if ((uint32_t)(raw >> 32) < tau) continue;
        const unsigned long long k = sort_key(raw);
        if ((k & pmask) == prefix) atomicAdd(&s_hist[(k >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t acc = 0, rank = s_rank;
        int d = 255;
        for (; d > 0; --d) {
          if (acc + s_hist[d] >= rank) break;
          acc += s_hist[d];
        }
        s_digit = (uint32_t)d;
        s_rank = rank - acc;
      }
      __syncthreads();
      prefix |= (unsigned long long)s_digit << shift;
      pmask |= 255ull << shift;
    }
    const unsigned long long kth = prefix;
    if (threadIdx.x == 0) s_n = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
      const unsigned long long raw = ck[i];
      if ((uint32_t)(raw >> 32) < tau) continue;
      const unsigned long long k = sort_key(raw);
      if (k >= kth) {
        const uint32_t p = atomicAdd(&s_n, 1u);
        if (p < kSelCap) {
          s_key[p] = k;
          s_slot[p] = (uint32_t)raw;
        }
      }
    }
    __syncthreads();
    m = min(s_n, (uint32_t)kSelCap);
  }
  const int n2 = pow2_at_least((int)(m ? m : 1));
  for (int i = (int)m + threadIdx.x; i < n2; i += blockDim.x) {
    s_key[i] = 0ull;
    s_slot[i] = 0xFFFFFFFFu;
  }
  __syncthreads();
  bitonic_desc(s_key, s_slot, n2);
  const uint32_t out = min(kp, m);
  for (uint32_t r = threadIdx.x; r < out; r += blockDim.x) {
    a.sel_key[(uint64_t)q * a.rmax + r] = s_key[r];
    a.sel_slot[(uint64_t)q * a.rmax + r] = s_slot[r];
  }
  if (threadIdx.x == 0) a.sel_cnt[q] = out;
  if (a.write_out) {
    const uint32_t kq = min(a.k[q], out);
    for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
      const bool ok = r < kq;
      const unsigned long long k = ok ? s_key[r] : 0ull;
      a.out_ids[(uint64_t)q * a.k_max + r] = ok ? 0xFFFFFFFFu - (uint32_t)k : 0xFFFFFFFFu;
      a.out_scores[(uint64_t)q * a.k_max + r] = ok ? key2f((uint32_t)(k >> 32)) : -INFINITY;
    }
    if (threadIdx.x == 0) {
      a.out_count[q] = kq;
      a.out_nmatch[q] = a.nmatch[q];
    }
  }
}

hipError_t launch_select(const SelectArgs& a, hipStream_t s) {
  if (!a.max_list) return hipSuccess;
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.cand_key);
  FR_REQUIRE(a.slot_ids);
  FR_REQUIRE(a.sel_key);
  FR_REQUIRE(a.sel_slot);
  FR_REQUIRE(a.sel_cnt);
  FR_REQUIRE(a.ovf);
  if (a.rmax > (uint32_t)kMaxR || a.rmax < 1) return hipErrorInvalidValue;
  if (a.write_out) {
    FR_REQUIRE(a.k);
    FR_REQUIRE(a.out_ids);
    FR_REQUIRE(a.out_scores);
    FR_REQUIRE(a.out_count);
    FR_REQUIRE(a.nmatch);
    FR_REQUIRE(a.out_nmatch);
  }
  hipLaunchKernelGGL(k_select, dim3(a.max_list), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------- rescore
// FP32 inner products of the selected candidates against the FP32 master
// rows (one wavefront per row, fixed lane split and reduction tree), then
// top-K by (FP32 score desc, id asc).
__global__ __launch_bounds__(256) void k_rescore(RescoreArgs a) {
  __shared__ unsigned long long s_key[kMaxR];
  const uint32_t q = blockIdx.x;
  if (q >= *a.n_dev) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (a.ovf[q]) {
    for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
      a.out_ids[(uint64_t)q * a.k_max + r] = 0xFFFFFFFFu;
      a.out_scores[(uint64_t)q * a.k_max + r] = -INFINITY;
    }
    if (threadIdx.x == 0) {
      a.out_count[q] = 0xFFFFFFFFu;
      a.out_nmatch[q] = a.nmatch[q];
    }
    return;
  }
  const uint32_t m = a.sel_cnt[q];
  const bool on = 4 * lane < (int)a.dpad;
  const float4 qv = on ? *((const float4*)(a.qrows + (uint64_t)q * a.dpad) + lane)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
  const unsigned long long* sk = a.sel_key + (uint64_t)q * a.rmax;
  const uint32_t* ss = a.sel_slot + (uint64_t)q * a.rmax;
  for (uint32_t r0 = wave * 4; r0 < m; r0 += 16) {
    float4 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t r = r0 + u;
      xv[u] = (on && r < m) ? *((const float4*)(a.master + (uint64_t)ss[r] * a.dpad) + lane)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float p = xv[u].x * qv.x;
      p = fmaf(xv[u].y, qv.y, p);
      p = fmaf(xv[u].z, qv.z, p);
      p = fmaf(xv[u].w, qv.w, p);
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) p += __shfl_xor(p, off);
      const uint32_t r = r0 + u;
      if (lane == 0 && r < m)
        s_key[r] = ((unsigned long long)fkey(p) << 32) | (sk[r] & 0xFFFFFFFFull);
    }
  }
  const int n2 = pow2_at_least((int)(m ? m : 1));
  for (int i = (int)m + threadIdx.x; i < n2; i += blockDim.x) s_key[i] = 0ull;
  __syncthreads();
  bitonic_desc(s_key, nullptr, n2);
  const uint32_t kq = min(a.k[q], m);
  for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
    const bool ok = r < kq;
    const unsigned long long k = ok ? s_key[r] : 0ull;
    a.out_ids[(uint64_t)q * a.k_max + r] = ok ? 0xFFFFFFFFu - (uint32_t)k : 0xFFFFFFFFu;
    a.out_scores[(uint64_t)q * a.k_max + r] = ok ? key2f((uint32_t)(k >> 32)) : -INFINITY;
  }
  if (threadIdx.x == 0) {
    a.out_count[q] = kq;
    a.out_nmatch[q] = a.nmatch[q];
  }
}

hipError_t launch_rescore(const RescoreArgs& a, hipStream_t s) {
  if (!a.max_q) return hipSuccess;
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.ovf);
  FR_REQUIRE(a.master);
  FR_REQUIRE(a.qrows);
  FR_REQUIRE(a.sel_key);
  FR_REQUIRE(a.sel_slot);
  FR_REQUIRE(a.sel_cnt);
  FR_REQUIRE(a.k);
  FR_REQUIRE(a.out_ids);
  FR_REQUIRE(a.out_scores);
  FR_REQUIRE(a.out_count);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.out_nmatch);
  if (a.rmax > (uint32_t)kMaxR || a.dpad > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rescore, dim3(a.max_q), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fr
