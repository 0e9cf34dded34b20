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
#include <float.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

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

// --------------------------------------------------- no-allocation scratch
// Device memory of the searches made through fr_search_noalloc: a fixed
// array in the code object, so that such a search needs no allocation.  Each
// device that loads the library holds its own copy until the process ends.
// On the host its name is only a stand-in: kernels get the device address
// that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
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
// Returns the row's L2 norm (in every lane).
template <int DT>
__device__ __forceinline__ float tile_row(const TileRowsArgs& a, uint64_t row, int lane) {
  constexpr int ES = DT == kF32 ? 4 : DT == kBF16 ? 2 : 1;
  constexpr int PC = 16 / ES;  // elements per 16-byte chunk
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
  const float nrm = sqrtf(ss);
  if (lane == 0) {
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
  return nrm;
}

template <int DT>
__global__ __launch_bounds__(256) void k_tile_rows(TileRowsArgs a) {
  const int lane = threadIdx.x & 63;
  const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  uint64_t n = a.n;
  if (a.n_dev) n = min(n, (uint64_t)*a.n_dev);
  if (row >= n) return;
  (void)tile_row<DT>(a, row, lane);
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

// ------------------------------------------------------------- prep
// One wavefront per query: the lanes clear its histogram, lane 0 sets the
// per-query state and builds the literal table.
__device__ __forceinline__ void prep_block0(const PrepArgs& a, uint32_t n_q) {
  if (blockIdx.x == 0 && threadIdx.x < kXcds) a.work[threadIdx.x] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.n_list = n_q;
    *a.n_list2 = 0u;
  }
}

// Per-query state of query q (one wavefront), given its norm.
__device__ __forceinline__ void prep_query(const PrepArgs& a, uint32_t q, int lane, float qn) {
  uint32_t* h = a.hist + (uint64_t)q * kHist;
  for (int i = lane; i < kHist; i += 64) h[i] = 0u;
  if (lane != 0) return;
  const uint32_t k = a.k[q];
  uint32_t kp = k;
  if (a.dt != kF32 && k) {
    kp = max(a.rescore_min, 4u * k);
    kp = min(kp, a.rescore_r);
    kp = max(kp, k);
  }
  a.kp[q] = kp;
  a.tau[q] = kp ? kKeyNegInf : kKeyPosInf;
  a.tsafe[q] = 0u;
  a.cnt[q] = 0u;
  a.smax[q] = 0u;
  a.nmatch[q] = 0ull;
  a.ovf[q] = 0u;
  a.qlist[q] = q;
  // histogram range [-|q| max|x|, +|q| max|x|] (Cauchy-Schwarz), so that
  // negative scores get buckets too; the starting-threshold kernel narrows
  // it to [starting threshold, hi] when it finds one
  const float m = __uint_as_float(*a.norm_max);
  const float hi = qn * m * 1.0001f;
  const bool rng_ok = hi > 0.f && isfinite(hi);
  a.hlo[q] = rng_ok ? -hi : 0.f;
  a.hinvw[q] = rng_ok ? (float)kNBF / (2.f * hi) : 0.f;
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
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const int lane = threadIdx.x & 63;
  const uint32_t q = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t n_q = *a.n_dev;
  prep_block0(a, n_q);
  if (q >= n_q || q >= a.max_q) return;
  prep_query(a, q, lane, a.qnorm[q]);
}

// The batch's query rows into the query tiles (norms, FP8 scales, the FP32
// copy the rescoring reads) and each query's per-search state, one
// wavefront per query.
template <int DT>
__global__ __launch_bounds__(256) void k_query_prep(TileRowsArgs t, PrepArgs a) {
  const int lane = threadIdx.x & 63;
  const uint32_t q = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t n_q = *a.n_dev;
  prep_block0(a, n_q);
  if (q >= n_q || q >= a.max_q || q >= t.n) return;
  const float qn = tile_row<DT>(t, q, lane);
  prep_query(a, q, lane, qn);
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.k);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.qnorm);
  FR_REQUIRE(a.norm_max);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.tsafe);
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
  hipLaunchKernelGGL(k_prep, dim3(grid_for(a.max_q ? a.max_q : 1, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_query_prep(const TileRowsArgs& t, const PrepArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.k);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.qnorm);
  FR_REQUIRE(a.norm_max);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.tsafe);
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
    FR_REQUIRE(t.rows);
  FR_REQUIRE(t.tiles);
  if (t.dt == kFP8) FR_REQUIRE(t.scale);
  if (t.dpad % 64 || t.dpad > 256 || t.dim > t.dpad || t.n_dev != a.n_dev || t.n != a.max_q)
    return hipErrorInvalidValue;
  const dim3 g(grid_for(a.max_q ? a.max_q : 1, 4)), b(256);
  switch (t.dt) {
    case kF32: hipLaunchKernelGGL(k_query_prep<kF32>, g, b, 0, s, t, a); break;
    case kBF16: hipLaunchKernelGGL(k_query_prep<kBF16>, g, b, 0, s, t, a); break;
    default: hipLaunchKernelGGL(k_query_prep<kFP8>, g, b, 0, s, t, a); break;
  }
  return hipGetLastError();
}


// Predicate masks of a search pass (Sec. 5.3: a document passes when every
// clause of the query's CNF has a term the document carries; with the live
// bits ANDed in).  Eight lanes build the 16 words of one (query, group): lane
// part p holds words 2p and 2p+1, so the live run and each literal's bitmap
// run (128 bytes) are read by one coalesced 16-byte load per lane.  A thread
// block covers 32 queries x gpt groups; the words are stored word-major so
// that the scan reads one word of consecutive queries from consecutive
// addresses.  Blocks go to the XCDs round robin: the blocks of one group
// range (all its query blocks) are given to the same XCD, so that the
// bitmap runs the queries share are read from HBM once into that XCD's L2.
__global__ __launch_bounds__(256) void k_mask_words(MaskWordArgs a) {
  if (a.run_if && *a.run_if == 0u) return;
  const uint32_t qx_n = (a.max_list + 31u) / 32u;          // query blocks
  const uint32_t idx = blockIdx.x / kXcds;
  const uint32_t gy = (idx / qx_n) * kXcds + blockIdx.x % kXcds;   // group range
  const uint32_t part = threadIdx.x & 7u;
  const uint32_t pos = (idx % qx_n) * 32u + (threadIdx.x >> 3);
  const uint32_t n = *a.n_list;
  if (pos >= n || pos >= a.max_list || (uint64_t)gy * a.gpt >= a.n_groups) return;
  const uint32_t q = a.qlist[pos];
  const uint32_t info = a.linfo[q];
  const bool empty = (info >> 24) & 1u, has = (info >> 26) & 1u, slow = (info >> 25) & 1u;
  const uint32_t nlit = info & 31u, starts = (info >> 8) & 0xFFFFu;
  uint32_t tl[kLits];
#pragma unroll
  for (int i = 0; i < kLits; ++i) tl[i] = a.lit[(uint64_t)q * kLits + i];
  const uint64_t g0 = (uint64_t)gy * a.gpt;
  const uint64_t g1 = min(g0 + a.gpt, (uint64_t)a.n_groups);
  unsigned long long cnt = 0;
  // words 2 part and 2 part + 1 of a 16-word run
  auto run2 = [&](const uint64_t* run) -> uint4 { return ((const uint4*)run)[part]; };
  const bool fast = !empty && has && !slow;
  for (uint64_t g = g0; g < g1; ++g) {
    uint64_t m0 = 0ull, m1 = 0ull;
    const uint64_t* gb = a.bits + g * (uint64_t)a.vocab * kWords;
    // the live run and every literal's run of the group, all loads in
    // flight at once
    uint4 lv = make_uint4(0u, 0u, 0u, 0u);
    uint4 lw[kLits];
    if (!empty) lv = run2(a.live + g * kWords);
#pragma unroll
    for (int i = 0; i < kLits; ++i)
      lw[i] = (fast && i < (int)nlit) ? run2(gb + (uint64_t)tl[i] * kWords)
                                      : make_uint4(0u, 0u, 0u, 0u);
    m0 = ((uint64_t)lv.y << 32) | lv.x;
    m1 = ((uint64_t)lv.w << 32) | lv.z;
    if (!empty && has) {
      uint64_t c0 = 0ull, c1 = 0ull;
      if (!slow) {
#pragma unroll
        for (int i = 0; i < kLits; ++i) {
          if (i < (int)nlit) {
            if (i > 0 && ((starts >> i) & 1u)) {
              m0 &= c0;
              m1 &= c1;
              c0 = c1 = 0ull;
            }
            c0 |= ((uint64_t)lw[i].y << 32) | lw[i].x;
            c1 |= ((uint64_t)lw[i].w << 32) | lw[i].z;
          }
        }
        m0 &= c0;
        m1 &= c1;
      } else {
        const uint32_t k0 = a.clause_off[q], k1 = a.clause_off[q + 1];
        for (uint32_t c = k0; c < k1; ++c) {
          c0 = c1 = 0ull;
          for (uint32_t l = a.literal_off[c]; l < a.literal_off[c + 1]; ++l) {
            const uint4 v = run2(gb + (uint64_t)a.terms[l] * kWords);
            c0 |= ((uint64_t)v.y << 32) | v.x;
            c1 |= ((uint64_t)v.w << 32) | v.z;
          }
          m0 &= c0;
          m1 &= c1;
        }
      }
    }
    a.mw[(g * kWords + 2 * part) * a.ppad + pos] = m0;
    a.mw[(g * kWords + 2 * part + 1) * a.ppad + pos] = m1;
    cnt += (unsigned long long)(__popcll(m0) + __popcll(m1));
  }
  // the query's eight lanes are consecutive: sum their counts
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) cnt += __shfl_xor(cnt, o);
  if (a.count_matches && part == 0 && cnt) atomicAdd(a.nmatch + q, cnt);
}
hipError_t launch_mask_words(const MaskWordArgs& a, hipStream_t s) {
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.live);
  FR_REQUIRE(a.bits);
  FR_REQUIRE(a.lit);
  FR_REQUIRE(a.linfo);
  FR_REQUIRE(a.clause_off);
  FR_REQUIRE(a.literal_off);
  FR_REQUIRE(a.terms);
  FR_REQUIRE(a.mw);
  FR_REQUIRE(a.nmatch);
  if (a.gpt < 1 || a.ppad < a.max_list || a.ppad % 256u) return hipErrorInvalidValue;
  if (a.max_list == 0 || a.n_groups == 0) return hipSuccess;
  // query blocks x group ranges, the ranges rounded up to whole XCD rounds
  const uint64_t gy_n = (a.n_groups + a.gpt - 1u) / a.gpt;
  const uint64_t blocks = (uint64_t)((a.max_list + 31u) / 32u) * ((gy_n + kXcds - 1) / kXcds) * kXcds;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mask_words, dim3((uint32_t)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// E4M3 (FN) code -> value
__device__ __forceinline__ float e4m3_to_f(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, m = b & 7u;
  const float v = e == 0u ? (float)m * 0.001953125f                       // m / 8 * 2^-6
                          : __uint_as_float(((e + 120u) << 23) | (m << 20));  // (1 + m/8) 2^(e-7)
  return (b & 0x80u) ? -v : v;
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
// chunks gives the dot products.  A chunks are read from LDS in groups of G,
// the next group's reads issued before the current group's matrix
// instructions (scheduling barriers keep that order), so LDS latency
// overlaps the matrix work.
// Products of the A chunks x[0 .. G) (chunks j0 .. j0 + G of the tile, in
// registers) with the matching chunks of every query block.
template <int DT, int CH, int QB, int G>
__device__ __forceinline__ void mma_chunks(f32x16 (&acc)[QB], const uint4 (&x)[G], int j0,
                                           const uint4 (&bq)[QB][CH]) {
    if constexpr (DT == kF32) {
      // 32x32x2 FP32: a chunk holds 4 consecutive k values per lane
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int j = j0 + i;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x[i].x), __uint_as_float(bq[b][j].x), acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x[i].y), __uint_as_float(bq[b][j].y), acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x[i].z), __uint_as_float(bq[b][j].z), acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x[i].w), __uint_as_float(bq[b][j].w), acc[b], 0, 0, 0);
        }
      }
    } else if constexpr (DT == kBF16) {
      // 32x32x16 BF16: one chunk = the 8 k values of one instruction
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int j = j0 + i;
#pragma unroll
        for (int b = 0; b < QB; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x[i]),
                                                            __builtin_bit_cast(bf16x8, bq[b][j]),
                                                            acc[b], 0, 0, 0);
      }
    } else {
      // 32x32x64 FP8 (E4M3, format code 0 for both operands, no block
      // scale): two chunks = the 32 k values of one instruction
#pragma unroll
      for (int i = 0; i < G; i += 2) {
        const int j = j0 + i;
        const i32x8 av = {(int)x[i].x, (int)x[i].y, (int)x[i].z, (int)x[i].w,
                          (int)x[i + 1].x, (int)x[i + 1].y, (int)x[i + 1].z, (int)x[i + 1].w};
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

// One tile's A chunks (chunk-major: chunk j of lane l at 1024 j + 16 l)
// from LDS into registers.
template <int CH>
__device__ __forceinline__ void lds_tile(uint4 (&x)[CH], const uint8_t* slot, int lane) {
  const uint4* p = (const uint4*)slot + lane;
#pragma unroll
  for (int j = 0; j < CH; ++j) x[j] = p[j * 64];
}

template <int DT, int CH, int QB>
__device__ __forceinline__ void mma_tile(f32x16 (&acc)[QB], const uint8_t* slot,
                                         const uint4 (&bq)[QB][CH], int lane) {
  const uint4* p = (const uint4*)slot + lane;
  // (FP32 with two query blocks: one chunk at a time, the B operand
  // already takes half the registers)
  constexpr int G = DT == kF32 ? (QB >= 2 ? 1 : 2) : (CH % 4 == 0 ? 4 : 2);
  constexpr int NG = CH / G;
  static_assert(CH % G == 0 && (DT != kFP8 || G % 2 == 0), "chunk groups");
  uint4 buf[2][G];
  auto load = [&](int g, uint4 (&d)[G]) {
#pragma unroll
    for (int i = 0; i < G; ++i) d[i] = p[(g * G + i) * 64];
  };
  auto work = [&](int g, const uint4 (&x)[G]) { mma_chunks<DT, CH, QB, G>(acc, x, g * G, bq); };
  load(0, buf[0]);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    __builtin_amdgcn_sched_barrier(0);
    if (g + 1 < NG) load(g + 1, buf[(g + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);
    work(g, buf[g & 1]);
  }
  __builtin_amdgcn_sched_barrier(0);
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
// Geometry of the scan's LDS ring.  A slot is one hand-over between the
// loader and the compute wavefronts: TPS consecutive tiles of one group
// (more documents per hand-over for the smaller tiles of the reduced
// precisions), the predicate-mask words of those tiles for the work item's
// QT queries ([word][QT] u64; a word covers two tiles), and for FP8 the
// tiles' row scales.
constexpr int kRingBytes = 112 * 1024;
template <int DT, int DPAD, int QT>
struct Ring {
  static constexpr int ES = DT == kF32 ? 4 : DT == kBF16 ? 2 : 1;
  static constexpr int CH = DPAD * ES / 32;   // 1 KB chunks per tile
  static constexpr int TB = CH * 1024;       // tile bytes
  static constexpr int TPS = TB > 16384 ? 1 : TB > 8192 ? 2 : 4;   // tiles per slot
  static constexpr int WPC = TPS >= 2 ? TPS / 2 : 1;               // mask words per slot
  static constexpr int LM = QT / 128;        // 1 KB loads per mask word
  static constexpr int MOFF = TPS * TB;      // offset of the mask words
  static constexpr int SOFF = MOFF + WPC * QT * 8;   // offset of the FP8 scales
  static constexpr int SB = SOFF + (DT == kFP8 ? TPS * kTile * 4 : 0);   // slot bytes
  static constexpr int LS = TPS * (CH + (DT == kFP8 ? 1 : 0)) + WPC * LM;   // loads per slot
  // slots in flight ahead of the one being scored: as many as the ring's
  // LDS share holds, within the 6-bit memory counter
  static constexpr int PDV = 63 / LS + 1;
  static constexpr int PDL = kRingBytes / SB - 1;
  static constexpr int PD = PDV < PDL ? PDV : PDL;
  static constexpr int NS = PD + 1;          // slots
  static_assert(PD >= 1 && (PD - 1) * LS <= 63, "ring geometry");
  static_assert(QT % 128 == 0 && SB % 16 == 0, "ring layout");
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

// LDS access written as inline assembly.  The loader wavefront uses these
// for its hand-over counters: the compiler cannot tell them apart from the
// ring its direct-to-LDS loads write, and would otherwise wait for every
// tile load in flight before each of them.  The read waits for itself only
// (four consecutive 16-byte aligned words in one read).
__device__ __forceinline__ uint4 lds_quad_ld(const uint32_t* p) {
  const uint32_t addr = (uint32_t)(size_t)(const __attribute__((address_space(3))) uint32_t*)p;
  uint4 v;
  __asm__ __volatile__("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr) : "memory");
  return v;
}
__device__ __forceinline__ void lds_word_st(uint32_t* p, uint32_t v) {
  const uint32_t addr = (uint32_t)(size_t)(__attribute__((address_space(3))) uint32_t*)p;
  __asm__ __volatile__("ds_write_b32 %0, %1" : : "v"(addr), "v"(v) : "memory");
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

// Wait until at most `younger` slots' loads of this wavefront are in flight.
template <int L, int PD>
__device__ __forceinline__ void wait_slots(uint32_t younger) {
  static_assert((PD - 1) * L <= 63, "memory counter range");
  switch (younger) {
    case 0: __builtin_amdgcn_s_waitcnt(vm_wait_code(0)); break;
    case 1: if constexpr (PD > 1) { __builtin_amdgcn_s_waitcnt(vm_wait_code(1 * L)); break; }
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

// Starting thresholds from a sample: the first a.n_groups groups of the
// corpus.  Step 1 scores every (sampled document, list position) pair with
// the scan's own tile product (one wavefront per kSeedTilesPerWave
// 32-document tiles and a 32-position query block, the same instruction
// sequence as the scan, so the scores match the scan's) and keeps, for every 16 documents of a tile
// (one lane's accumulator rows), the two best matching scores: a subset of
// the sample's matches.  Step 2 reads two ranks off each query's subset
// through a histogram of its scores:
//   * the K'-th best, a lower bound of the K'-th best match of the corpus
//     (the K'-th best of any subset of the matches is at most the K'-th
//     best of all of them): the safe start;
//   * the r-th best for the r of kSpecL (the speculative start, used when
//     r < K'): below the corpus's K'-th best except with probability about
//     10^-4 by the bound, about 10^-6 in fact; if a pass collects fewer than
//     min(K', n_match) candidates from it, the query is scanned again from
//     the safe start, so the result stays exact.
// Both are read from bucket edges and lowered by twice the FP32 summation
// bound gamma_d * |q| * max|x| (12.5 % slack for the quantised forms'
// scaled norms), so they stay lower bounds whatever the accumulation order.
template <int DT, int DPAD>
__global__ __launch_bounds__(256) void k_seed_scores(SeedArgs a) {
  constexpr int ES = DT == kF32 ? 4 : DT == kBF16 ? 2 : 1;
  constexpr int CH = DPAD * ES / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const uint32_t n_list = *a.n_list;
  const uint32_t pos0 = blockIdx.y * (uint32_t)kTile;
  const uint32_t ng = a.n_groups;
  const uint32_t n_t = ng * (uint32_t)(kGroup / kTile);
  const uint32_t t0 = (blockIdx.x * 4u + (uint32_t)wave) * kSeedTilesPerWave;
  if (pos0 >= n_list || pos0 >= a.max_list || t0 >= n_t) return;
  const uint32_t pos = pos0 + (uint32_t)col;
  const bool qv = pos < n_list && pos < a.max_list;
  const uint32_t q = qv ? a.qlist[pos] : 0u;
  // the query block's B operand, loaded once for the wavefront's tiles
  uint4 bq[1][CH];
  const uint4* qp = (const uint4*)(a.qtiles + (uint64_t)(q / kTile) * (CH * 1024)) + half * 32 +
                    (q % kTile);
#pragma unroll
  for (int j = 0; j < CH; ++j) bq[0][j] = qv ? qp[j * 64] : make_uint4(0, 0, 0, 0);
  const float qs = DT == kFP8 && qv ? a.qscale[q] : 1.f;
  // the two best keys among this lane's matching rows of tile t (0: none),
  // from its products, the query's mask word of the tile (tile t is tile
  // t % 32 of group t / 32: half of mask word (t % 32) / 2) and, for FP8,
  // the lane's row scales (rows 8g + 4 half .. + 3 in xs[g])
  auto keep_two = [&](uint32_t t, const f32x16& acc, uint64_t mword, const float4 (&xs)[4]) {
    const uint32_t tg = t % (uint32_t)(kGroup / kTile);
    const uint32_t mrow = (uint32_t)(mword >> ((tg & 1u) * 32u)) >> (4 * half);
    uint32_t k1 = 0u, k2 = 0u;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float sc = acc[v];
      if constexpr (DT == kFP8) {
        const float4 x4 = xs[v >> 2];
        sc = (sc * qs) * ((v & 3) == 0 ? x4.x : (v & 3) == 1 ? x4.y : (v & 3) == 2 ? x4.z : x4.w);
      }
      const uint32_t key = ((mrow >> (8 * (v >> 2) + (v & 3))) & 1u) ? fkey(sc) : 0u;
      const uint32_t lo = min(k1, key);
      k1 = max(k1, key);
      k2 = max(k2, lo);
    }
    *(uint2*)(a.skey + (uint64_t)pos * a.row + (uint64_t)t * 4u + 2u * (uint32_t)half) =
        make_uint2(k1, k2);
  };
  auto mask_word = [&](uint32_t t) -> uint64_t {
    return a.mw[((uint64_t)(t / (uint32_t)(kGroup / kTile)) * kWords +
                 (t % (uint32_t)(kGroup / kTile)) / 2u) * a.ppad + pos];
  };
  if constexpr (DT == kF32) {
    const float4 none[4] = {};
    for (uint32_t t = t0; t < min(t0 + kSeedTilesPerWave, n_t); ++t) {
      f32x16 acc[1];
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[0][v] = 0.f;
      mma_tile<DT, CH, 1>(acc, a.tiles + (uint64_t)t * (CH * 1024), bq, lane);
      if (qv) keep_two(t, acc[0], mask_word(t), none);
    }
  } else {
    // BF16/FP8: every tile's A operand, mask word and row scales are loaded
    // at once, with the query operand (one round of memory latency), then
    // the tiles are scored with the scan's instruction sequence
    constexpr int TPW = (int)kSeedTilesPerWave;
    uint4 av[TPW][CH];
    uint64_t mwd[TPW];
    float4 xs[TPW][4];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const uint32_t t = t0 + (uint32_t)i;
      const uint32_t tl = t < n_t ? t : t0;                 // an existing tile
      const uint4* p = (const uint4*)(a.tiles + (uint64_t)tl * (CH * 1024)) + lane;
#pragma unroll
      for (int j = 0; j < CH; ++j) av[i][j] = p[j * 64];
      mwd[i] = (qv && t < n_t) ? mask_word(t) : 0ull;
      if constexpr (DT == kFP8) {
        const float4* s = (const float4*)(a.xscale + (uint64_t)tl * kTile) + half;
#pragma unroll
        for (int g = 0; g < 4; ++g) xs[i][g] = s[2 * g];
      }
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const uint32_t t = t0 + (uint32_t)i;
      if (t >= n_t) break;
      f32x16 acc[1];
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[0][v] = 0.f;
      mma_chunks<DT, CH, 1, CH>(acc, av[i], 0, bq);
      if (qv) keep_two(t, acc[0], mwd[i], xs[i]);
    }
  }
}

// Bucket of a per-query histogram (kSeedBins counters, lane l holding
// buckets 32 l .. 32 l + 31 in c) where the count from the top first
// reaches `rank`; -1 if the histogram holds fewer.  Wave-uniform.
__device__ __forceinline__ int seed_rank_bucket(const uint32_t (&c)[32], uint32_t lane_sum,
                                                uint32_t suffix_incl, uint32_t rank, int lane) {
  const uint32_t above = suffix_incl - lane_sum;   // counts in higher lanes
  int found = -1;
  if (rank > 0u && above < rank && rank <= suffix_incl) {
    uint32_t run = above;
    for (int e = 31; e >= 0; --e) {
      run += c[e];
      if (run >= rank) {
        found = 32 * lane + e;
        break;
      }
    }
  }
  const uint64_t bal = __ballot(found >= 0);     // one lane at most
  if (!bal) return -1;
  return __shfl(found, __builtin_ctzll(bal));
}

// One workgroup per list position: the kept sample scores go into a
// histogram of kSeedBins buckets over [-|q| max|x|, +|q| max|x|] in LDS (the
// paper's bucket top-K, appendix "Fast Top K Selection", with the
// Cauchy-Schwarz range standing in for the known score bounds); each
// starting threshold is the lower edge of the bucket below the one where its
// rank is reached, so it is at most the rank's score.  The scan's histogram
// range is narrowed to [start, |q| max|x|].
constexpr int kSeedSelThreads = 256;
__global__ __launch_bounds__(kSeedSelThreads) void k_seed_select(SeedArgs a) {
  __shared__ uint32_t s_hist[kSeedBins];
  __shared__ uint32_t s_ms;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t pos = blockIdx.x;
  if (pos >= *a.n_list || pos >= a.max_list) return;
  const uint32_t q = a.qlist[pos];
  const uint32_t kp = a.kp[q];
  const float bound = a.qnorm[q] * __uint_as_float(*a.norm_max);
  const float hi = bound * 1.0001f;
  if (kp == 0u || !(hi > 0.f) || !isfinite(hi)) return;
  const float w = (float)kSeedBins / (2.f * hi);
  for (int i = tid; i < kSeedBins; i += kSeedSelThreads) s_hist[i] = 0u;
  if (tid == 0) s_ms = 0u;
  __syncthreads();
  // the kept scores (key 0: none) and the sample's matches
  const uint32_t n = a.n_groups * (uint32_t)(kGroup / kTile) * 4u;
  const uint4* src = (const uint4*)(a.skey + (uint64_t)pos * a.row);
  for (uint32_t i = (uint32_t)tid; i < n / 4u; i += kSeedSelThreads) {
    const uint4 v = src[i];
    const uint32_t k4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (!k4[e]) continue;
      const float fb = (key2f(k4[e]) + hi) * w;
      const int bk = fb >= (float)(kSeedBins - 1) ? kSeedBins - 1 : (fb > 0.f ? (int)fb : 0);
      atomicAdd(&s_hist[bk], 1u);
    }
  }
  uint32_t ms = 0u;
  for (uint32_t i = (uint32_t)tid; i < a.n_groups * (uint32_t)kWords; i += kSeedSelThreads)
    ms += (uint32_t)__popcll(a.mw[(uint64_t)i * a.ppad + pos]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) ms += __shfl_xor(ms, off);
  if (lane == 0 && ms) atomicAdd(&s_ms, ms);
  __syncthreads();
  if (tid >= 64) return;
  ms = s_ms;
  uint32_t c[32], sum = 0u;
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    c[e] = s_hist[32 * lane + e];
    sum += c[e];
  }
  // inclusive suffix sum over lanes (higher lanes hold higher scores)
  uint32_t suf = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_down(suf, off, 64);
    if (lane + off < 64) suf += o;
  }
  // speculative rank from the Bernstein bound (see kSpecL), p = the share
  // of the query's matches that lie in the sample
  uint32_t r = kp;
  const double m_all = (double)a.nmatch[q];
  if (m_all > 0.0 && ms > 0u && !(a.strategy & kStratNoSpec)) {
    const float p = fminf(1.f, (float)((double)ms / m_all));
    const float mu = (float)kp * p;
    const float l3 = 2.f * kSpecL / 3.f;
    const float t = 0.5f * (l3 + sqrtf(l3 * l3 + 8.f * kSpecL * mu));
    const float rf = floorf(mu + t) + 1.f;
    if (rf < (float)kp) r = (uint32_t)rf;
  }
  const int b_safe = seed_rank_bucket(c, sum, suf, kp, lane);
  const int b_spec = r < kp ? seed_rank_bucket(c, sum, suf, r, lane) : -1;
  if (lane != 0) return;
  const float u = 5.9604644775390625e-8f;   // 2^-24
  const float dd = (float)a.dim;
  const float gam = dd * u / (1.f - dd * u);
  const float tol = 2.f * gam * bound * 1.125f + 1e-30f;
  auto edge = [&](int b) -> float { return -hi + (float)(b - 1) / w - tol; };
  const float t_safe = b_safe >= 0 ? edge(b_safe) : -INFINITY;
  const float t_spec = b_spec >= 0 ? edge(b_spec) : -INFINITY;
  const float start = fmaxf(t_safe, t_spec);
  if (!(start > -INFINITY)) return;            // too few matches in the sample
  atomicMax(a.tau + q, fkey(start));
  a.tsafe[q] = start > t_safe ? fkey(t_safe) : 0u;
  // every candidate of the scan scores at least `start`: the histogram
  // range shrinks to [start, hi], so its buckets are finer
  if (start < hi) {
    a.hlo[q] = start;
    a.hinvw[q] = (float)kNBF / (hi - start);
  }
}

#define FR_SEED_CASES(X) \
  X(kF32, 64) X(kF32, 128) X(kF32, 192) X(kF32, 256) \
  X(kBF16, 64) X(kBF16, 128) X(kBF16, 192) X(kBF16, 256) \
  X(kFP8, 64) X(kFP8, 128) X(kFP8, 192) X(kFP8, 256)

hipError_t launch_seed(const SeedArgs& a, int dt, int dpad, hipStream_t s) {
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.kp);
  FR_REQUIRE(a.tiles);
  FR_REQUIRE(a.qtiles);
  FR_REQUIRE(a.qnorm);
  FR_REQUIRE(a.norm_max);
  FR_REQUIRE(a.mw);
  FR_REQUIRE(a.skey);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.tau);
  FR_REQUIRE(a.tsafe);
  FR_REQUIRE(a.hlo);
  FR_REQUIRE(a.hinvw);
  if (dt == kFP8) {
    FR_REQUIRE(a.xscale);
    FR_REQUIRE(a.qscale);
  }
  if (a.max_list == 0 || a.n_groups == 0) return hipSuccess;
  if (a.ppad < a.max_list) return hipErrorInvalidValue;
  // four kept keys per sampled tile, all of them held in LDS by the select
  if ((uint64_t)a.n_groups * (kGroup / kTile) * 4u > a.row || a.row % 4u ||
      (uint64_t)a.n_groups * (kGroup / kTile) * 4u > (uint64_t)kSeedKeysMax)
    return hipErrorInvalidValue;
  const uint32_t ng = a.n_groups;
  const dim3 g1((ng * (kGroup / kTile) + 4u * kSeedTilesPerWave - 1u) / (4u * kSeedTilesPerWave),
                (a.max_list + kTile - 1u) / kTile);
#define FR_SEED(D, P)                                                  \
  if (dt == D && dpad == P) {                                          \
    hipLaunchKernelGGL((k_seed_scores<D, P>), g1, dim3(256), 0, s, a); \
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;   \
    hipLaunchKernelGGL(k_seed_select, dim3(a.max_list), dim3(kSeedSelThreads), 0, s, a); \
    return hipGetLastError();                                          \
  }
  FR_SEED_CASES(FR_SEED)
#undef FR_SEED
  return hipErrorInvalidValue;
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
//     LDS ring, up to PD tiles ahead, and publishes each slot once its
//     direct-to-LDS loads have landed; with them it copies the predicate
//     masks of the item's queries (computed beforehand by k_mask_words) for
//     the next group;
//   * compute wavefront w owns QB blocks of 32 queries (B operand in
//     registers).  Per tile it scores the tile on the matrix cores (unless
//     no query of it matches the tile), drops (doc, query) pairs that fail
//     the predicate mask or score below the query's threshold, and appends
//     the rest to its staging ring in LDS;
//   * the keeper wavefront, on a fixed clock period, moves staged candidates
//     to the global per-query buffers and histograms (space reserved in one
//     period, entries written in the next) and raises the thresholds from
//     the global histograms (one pipeline stage per period, so every load
//     it waits for is a period old).  Compute wavefronts read the
//     thresholds from LDS at every tile.
// The three kinds of wavefront hand over work through counters in LDS
// (slot published, tiles done, staging head and tail, item finished), so a
// slow tile or a long memory round trip in one of them does not stall the
// others; the ring and the staging rings absorb the difference.  Compute
// wavefronts issue no global atomics in the tile loop unless their staging
// ring is full (then they append directly).  All wavefronts meet at
// workgroup barriers only between items: two per item fetch, one after the
// item set-up, one at the item end.
template <int DT, int DPAD, int QB, int NW>
__global__ __launch_bounds__((NW + 2) * 64) void k_scan(ScanArgs a) {
  constexpr int QT = NW * QB * 32;          // queries per work item
  using R = Ring<DT, DPAD, QT>;
  constexpr int CH = R::CH;                 // 16-byte chunks per lane per tile
  constexpr int TPS = R::TPS;               // tiles per ring slot
  constexpr int PD = R::PD;                 // slots in flight
  constexpr int NS = R::NS;                 // ring slots
  constexpr int SR = NW > 4 ? 256 : 512;    // staging ring entries per wavefront
  constexpr long long kPeriod = 3000;       // keeper period, shader clocks
  constexpr int RJ = QT / 64;               // queries per keeper lane
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  static_assert(QT <= 256, "staged query index is one byte");
  static_assert(NW % 4 == 0, "done counters are read four at a time");
  __shared__ __attribute__((aligned(16))) uint8_t s_ring[NS * R::SB];
  __shared__ uint32_t s_item;
  // per query of the item, index j = (wave * QB + b) * 32 + col
  __shared__ float s_thr[QT];
  __shared__ uint32_t s_qg[QT];             // batch query index, kNone if unused
  __shared__ uint32_t s_qkp[QT];            // selection size
  __shared__ float s_qlo[QT];
  __shared__ float s_qiw[QT];
  // ring hand-over: sequence number of the slot load in each slot, slot
  // loads done per compute wavefront (sequence numbers run on across items)
  __shared__ uint32_t s_ready[NS];
  __shared__ __attribute__((aligned(16))) uint32_t s_done[NW];
  __shared__ uint32_t s_fin[NW];            // item number a compute wavefront finished
  // staging rings: entries (score key << 32 | slot) and the query's j;
  // head written by the compute wavefront, tail by the keeper
  __shared__ unsigned long long s_sk[NW][SR];
  __shared__ uint8_t s_sq[NW][SR];
  __shared__ uint32_t s_shead[NW];
  __shared__ uint32_t s_stail[NW];
  // keeper scratch
  __shared__ uint32_t s_hcnt[QT];
  __shared__ uint32_t s_hcur[QT];
  __shared__ uint32_t s_hbase[QT];
  __shared__ uint32_t s_hmax[QT];
  __shared__ uint32_t s_dirty[QT / 32];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5,
            col = lane & 31;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t n_list = *a.n_list;
  const uint32_t n_qtiles = (n_list + QT - 1) / QT;
  const uint64_t n_tiles = (uint64_t)a.n_groups * (kGroup / kTile);
  const uint32_t n_chunks = (uint32_t)((n_tiles + a.tpi - 1) / a.tpi);
  const uint32_t my_chunks = n_chunks > xcd ? (n_chunks - xcd + kXcds - 1) / kXcds : 0u;
  const uint32_t my_items = my_chunks * n_qtiles;
  // the item's tiles [t0, t1) (identical in every wavefront; t0 and the
  // count are multiples of 4, so of TPS)
  auto item_range = [&](uint32_t item, uint64_t& t0, uint64_t& t1) {
    const uint32_t chunk = (item / n_qtiles) * kXcds + xcd;
    t0 = (uint64_t)chunk * a.tpi;
    t1 = min(t0 + a.tpi, n_tiles);
  };
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // LDS word written by another wavefront of the workgroup; the hand-over
  // counters are one value for the whole wavefront, so the result is made
  // wave-uniform (scalar loop control in the waits)
  auto lds_get = [](const uint32_t* p) -> uint32_t {
    return __builtin_amdgcn_readfirstlane(__atomic_load_n(p, __ATOMIC_RELAXED));
  };
  auto lds_put = [](uint32_t* p, uint32_t v) {
    __asm__ __volatile__("" ::: "memory");     // earlier LDS accesses first
    __atomic_store_n(p, v, __ATOMIC_RELAXED);
  };

  if (wave == NW) {
    // ---------------------------------------------------------- loader
    // Slot load seq (TPS tiles, their mask words and FP8 scales) goes to
    // slot seq % NS.  It is issued once every compute wavefront is done with
    // the slot's previous load (seq - NS) and fewer than PD loads are in
    // flight; the oldest load in flight is published (the slot's sequence
    // number set) once its data have landed.  Every slot load is the same
    // R::LS instructions, so the memory counter tells which have landed.
    uint32_t seq0 = 0;                                // first slot load of the item
    for (;;) {
      wg_barrier();
      const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
      wg_barrier();
      if (item >= my_items) break;
      uint64_t t0, t1;
      item_range(item, t0, t1);
      const uint32_t n_s = (uint32_t)((t1 - t0) / TPS);
      const uint32_t qt = item % n_qtiles;
      // slot load c: tiles t0 + c*TPS .. of the item and their mask words
      // (word w of group g, 64 documents, is word g*kWords + w = tile / 2 of
      // the pass)
      auto dma_slot = [&](uint32_t c, uint8_t* sp) {
        const uint64_t tile = t0 + (uint64_t)c * TPS;
#pragma unroll
        for (int u = 0; u < TPS; ++u)
          dma_tile<DT, CH>(a.tiles, a.xscale, tile + u, sp + u * R::TB,
                           (float*)(sp + R::SOFF) + u * kTile, lane);
#pragma unroll
        for (int wl = 0; wl < R::WPC; ++wl) {
          const uint64_t* src = a.mw + (tile / 2 + wl) * a.ppad + (uint64_t)qt * QT + 2u * lane;
#pragma unroll
          for (int k = 0; k < R::LM; ++k)
            __builtin_amdgcn_global_load_lds(
                (const void*)(src + 128 * k),
                (__attribute__((address_space(3))) void*)(sp + R::MOFF + wl * QT * 8 + 1024 * k),
                16, 0, 0);
        }
      };
      wg_barrier();                                   // set-up
      uint32_t issued = 0, published = 0;
      // least done-counter over the compute wavefronts as last read: the
      // counters only grow, so a slot it shows free is free
      uint32_t mind = 0;
      while (published < n_s) {
        bool moved = false;
        while (issued < n_s && issued - published < (uint32_t)PD) {
          const uint32_t sq = seq0 + issued;
          if (sq >= (uint32_t)NS && mind < sq - (uint32_t)NS + 1u) {
            uint32_t m = 0xFFFFFFFFu;
#pragma unroll
            for (int w = 0; w < NW; w += 4) {
              const uint4 d = lds_quad_ld(&s_done[w]);
              m = min(m, min(min(d.x, d.y), min(d.z, d.w)));
            }
            mind = __builtin_amdgcn_readfirstlane(m);
            if (mind < sq - (uint32_t)NS + 1u) break;   // slot still in use
          }
          dma_slot(issued, s_ring + (sq % (uint32_t)NS) * R::SB);
          ++issued;
          moved = true;
        }
        if (published < issued) {
          wait_slots<R::LS, PD>(issued - published - 1u);
          const uint32_t sq = seq0 + published;
          if (lane == 0) lds_word_st(&s_ready[sq % (uint32_t)NS], sq);
          ++published;
          moved = true;
        }
        if (!moved) __builtin_amdgcn_s_sleep(1);
      }
      seq0 += n_s;
      wg_barrier();                                   // item end
    }
    return;
  }

  if (wave == NW + 1) {
    // ---------------------------------------------------------- keeper
    // Moving staged entries to the global buffers takes two periods: count
    // the new entries per query and reserve global space (one atomic per
    // query, whose result is used a period later), then scatter them, add
    // their histogram buckets and raise the running maximum.
    uint32_t rbase[RJ];           // reserved global position, per query of the lane
    uint32_t rres = 0;            // bit r: rbase[r] is pending
    bool pend = false;            // entries [p0, p1) of every ring are reserved
    uint32_t p0[NW], p1[NW];
    auto count_reserve = [&]() {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        p0[w] = lds_get(&s_stail[w]);
        p1[w] = lds_get(&s_shead[w]);
        for (uint32_t i = p0[w] + lane; i < p1[w]; i += 64)
          atomicAdd(&s_hcnt[s_sq[w][i % SR]], 1u);
      }
      wave_sync();
      rres = 0;
#pragma unroll
      for (int r = 0; r < RJ; ++r) {
        const int j = lane + 64 * r;
        const uint32_t c = s_hcnt[j];
        if (c) {
          rbase[r] = atomicAdd(a.cnt + s_qg[j], c);
          rres |= 1u << r;
          atomicOr(&s_dirty[j >> 5], 1u << (j & 31));
        }
        s_hcnt[j] = 0u;
      }
      pend = true;
      wave_sync();
    };
    auto scatter = [&]() {
#pragma unroll
      for (int r = 0; r < RJ; ++r)
        if ((rres >> r) & 1u) s_hbase[lane + 64 * r] = rbase[r];
      wave_sync();
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        for (uint32_t i = p0[w] + lane; i < p1[w]; i += 64) {
          const uint32_t j = s_sq[w][i % SR];
          const unsigned long long key = s_sk[w][i % SR];
          const uint32_t r = atomicAdd(&s_hcur[j], 1u);
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
        s_hcur[j] = 0u;
      }
      // the entries are consumed: hand their ring space back
      if (lane < NW) {
#pragma unroll
        for (int w = 0; w < NW; ++w)
          if (w == lane) lds_put(&s_stail[w], p1[w]);
      }
      rres = 0;
      pend = false;
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
      if (a.strategy & kStratNoRefresh) return;   // thresholds stay at their start
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

    uint32_t item_no = 0;
    for (;;) {
      wg_barrier();
      const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
      wg_barrier();
      if (item >= my_items) break;
      wg_barrier();                                   // set-up: s_qg, s_thr valid
      for (int i = lane; i < QT / 32; i += 64) s_dirty[i] = 0u;
      for (int j = lane; j < QT; j += 64) {
        s_hcnt[j] = 0u;
        s_hcur[j] = 0u;
        s_hmax[j] = 0u;
      }
      rstage = 0;
      pend = false;
      rres = 0;
      wave_sync();
      long long last = (long long)__builtin_readcyclecounter();
      for (uint32_t period = 1;; ++period) {
        // wait for the next period (or the end of the item's tiles)
        bool fin;
        for (;;) {
          fin = true;
#pragma unroll
          for (int w = 0; w < NW; ++w) fin = fin && lds_get(&s_fin[w]) == item_no;
          if (fin || (long long)__builtin_readcyclecounter() - last >= kPeriod) break;
          __builtin_amdgcn_s_sleep(2);
        }
        last = (long long)__builtin_readcyclecounter();
        refresh_consume();
        if (pend) scatter();
        count_reserve();
        if (fin) {
          // every compute wavefront is done with the item: move the rest
          scatter();
          if (rstage == 2) refresh_issue();
          refresh_drain();
          break;
        }
        refresh_issue();
      }
      ++item_no;
      wg_barrier();                                   // item end
    }
    return;
  }

  // ------------------------------------------------------------ compute
  // the wavefront's own entries of the hand-over arrays, addressed from a
  // scalar copy of its index (a vector copy kept live across the loops is
  // what the register allocator spills)
  auto wave_s = [&]() -> int { return __builtin_amdgcn_readfirstlane(wave); };
  constexpr int NQW = 32 * QB;              // queries per wavefront
  // matrix-core B operand and per-query state, block b -> query column col
  uint4 bq[QB][CH];
  uint32_t qi[QB], kp[QB];
  float thr[QB], hlo[QB], hinv[QB], qs[QB];
  bool qv[QB];
  if (wave == 0) {
    for (int i = lane; i < NS; i += 64) s_ready[i] = 0xFFFFFFFFu;
    for (int i = lane; i < NW; i += 64) {
      s_done[i] = 0u;
      s_fin[i] = 0xFFFFFFFFu;
      s_shead[i] = 0u;
      s_stail[i] = 0u;
    }
  }
  uint32_t seq0 = 0;            // sequence number of the item's first slot load
  uint32_t item_no = 0;
  uint32_t shead = 0;           // this wavefront's staging head (it is the only writer)

  // Query-block sharing: when the query tile fills only nb of the NW
  // wavefronts' blocks (a small batch) and nb divides NW, wavefront w takes
  // block w % nb and the tiles t with t % (NW / nb) == w / nb, so that every
  // wavefront does matrix work; each (query, tile) pair is still scored once.
  int bw = wave;                // block of queries this wavefront holds
  uint32_t tstride = 1, tslot = 0;
  auto my_pos = [&](uint32_t qt, int b) -> uint32_t {
    return qt * QT + (uint32_t)((bw * QB + b) * 32 + col);
  };
  auto my_j = [&](int b) -> int { return (bw * QB + b) * 32 + col; };
  auto load_queries = [&](uint32_t qt) {
    const uint32_t valid = min((uint32_t)QT, n_list - qt * (uint32_t)QT);
    const uint32_t nb = (valid + 32u * QB - 1u) / (32u * QB);
    if (nb < (uint32_t)NW && (uint32_t)NW % nb == 0u) {
      bw = wave % (int)nb;
      tstride = (uint32_t)NW / nb;
      tslot = (uint32_t)wave / nb;
    } else {
      bw = wave;
      tstride = 1;
      tslot = 0;
    }
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
        // every wavefront writes the state of its own block: the block it
        // holds, or (when it shares another block) an unused one
        const int j = (wave * QB + b) * 32 + col;
        const bool own = bw == wave;
        s_qg[j] = (own && qv[b] && kp[b]) ? q : kNone;
        s_qkp[j] = own ? kp[b] : 0u;
        s_qlo[j] = own ? hlo[b] : 0.f;
        s_qiw[j] = own ? hinv[b] : 0.f;
        s_thr[j] = own ? thr[b] : INFINITY;
      }
      const uint4* p = (const uint4*)(a.qtiles + (uint64_t)(q / kTile) * (CH * 1024)) +
                       half * 32 + (q % kTile);
#pragma unroll
      for (int j = 0; j < CH; ++j) bq[b][j] = qv[b] ? p[j * 64] : make_uint4(0, 0, 0, 0);
    }
  };

  // ------------------------------------------------------------ items
  uint32_t cur_qt = 0xFFFFFFFFu;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.work + xcd, 1u);
    wg_barrier();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
    wg_barrier();
    if (item >= my_items) break;
    const uint32_t qt = item % n_qtiles;
    uint64_t t0, t1;
    item_range(item, t0, t1);

    if (qt != cur_qt) {
      cur_qt = qt;
      load_queries(qt);
    }
    wg_barrier();                                     // set-up

    const uint32_t n_s = (uint32_t)((t1 - t0) / TPS);
#pragma unroll 1
    for (uint32_t c = 0; c < n_s; ++c) {
      // one step per ring slot: wait until the loader has published it,
      // then score each of its tiles that a query of this wavefront matches
      const uint32_t sq = seq0 + c;
      const uint32_t rs = sq % (uint32_t)NS;
      while (lds_get(&s_ready[rs]) != sq) __builtin_amdgcn_s_sleep(1);
      const uint8_t* sp = s_ring + rs * R::SB;
      const uint64_t* smw = (const uint64_t*)(sp + R::MOFF);   // [word][QT]
      // the lane's query column, worked out again for every slot: kept live
      // across the whole loop it is the value the register allocator spills
      // (a scratch reload per slot)
      uint32_t lid = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
      __asm__ __volatile__("" : "+v"(lid));
      const int bws = __builtin_amdgcn_readfirstlane(bw);
      auto slot_j = [&](int b) -> int { return (bws * QB + b) * 32 + (int)(lid & 31u); };
      const uint64_t tile0 = t0 + (uint64_t)c * TPS;            // the slot's first tile
      const uint32_t tg0 = (uint32_t)(tile0 % (kGroup / kTile));   // ... within its group
      // the slot's mask words of this wavefront's queries (kept in registers
      // for the epilogues); bit u of act: tile u of the slot has a match for
      // some query of this wavefront
      uint64_t mwv[QB][R::WPC];
      uint32_t act = 0;
#pragma unroll
      for (int wl = 0; wl < R::WPC; ++wl) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          mwv[b][wl] = kp[b] ? smw[wl * QT + slot_j(b)] : 0ull;
          o |= mwv[b][wl];
        }
        if constexpr (TPS == 1) {
          if (__ballot((uint32_t)(o >> ((tg0 & 1u) * 32u)) != 0u)) act = 1u;
        } else {
          if (__ballot((uint32_t)o != 0u)) act |= 1u << (2 * wl);
          if (__ballot((uint32_t)(o >> 32) != 0u)) act |= 2u << (2 * wl);
        }
      }
      if (act) {
#pragma unroll
        for (int b = 0; b < QB; ++b) thr[b] = s_thr[slot_j(b)];
      }
      // the staging ring's tail as of now (it only advances, so the room
      // computed from it is a lower bound)
      const uint32_t tail0 = __atomic_load_n(&s_stail[wave_s()], __ATOMIC_RELAXED);
      // bit u: this wavefront scores tile u of the slot
      uint32_t todo = 0;
#pragma unroll
      for (int u = 0; u < TPS; ++u)
        if (((act >> u) & 1u) && (tg0 + (uint32_t)u) % tstride == tslot) todo |= 1u << u;
      // BF16/FP8: a whole tile's A operand fits in registers, so the next
      // tile's is read from LDS while this tile's products and epilogue run
      constexpr bool kPre = DT != kF32;
      uint4 abuf[kPre ? CH : 1];
      if constexpr (kPre) {
        if (todo) lds_tile<CH>(abuf, sp + __builtin_ctz(todo) * R::TB, lane);
      }
#pragma unroll
      for (int u = 0; u < TPS; ++u) {
        const uint32_t t = tg0 + (uint32_t)u;                 // tile within its group
        const int wl = TPS == 1 ? 0 : u / 2;                  // its mask word in the slot
        if (!((todo >> u) & 1u)) continue;
        f32x16 accs[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) accs[b][v] = 0.f;
        if constexpr (kPre) {
          mma_chunks<DT, CH, QB, CH>(accs, abuf, 0, bq);
          const uint32_t nxt = todo & ~((2u << u) - 1u);
          if (nxt) lds_tile<CH>(abuf, sp + __builtin_ctz(nxt) * R::TB, lane);
        } else {
          mma_tile<DT, CH, QB>(accs, sp + u * R::TB, bq, lane);
        }
        float4 xs[4];
        if constexpr (DT == kFP8) read_scales(xs, (const float*)(sp + R::SOFF) + u * kTile, lane);
#pragma unroll
        for (int b = 0; b < QB; ++b) {
          f32x16& acc = accs[b];
          const uint32_t m32 = (uint32_t)(mwv[b][wl] >> ((t & 1u) * 32u));
          if constexpr (DT == kFP8) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float4 x4 = xs[v >> 2];
              const float sc = (v & 3) == 0 ? x4.x : (v & 3) == 1 ? x4.y : (v & 3) == 2 ? x4.z : x4.w;
              acc[v] = (acc[v] * qs[b]) * sc;
            }
          }
          // rows that fail the predicate become -inf: a row's mask bit
          // (row 8g + 4 half + i = acc_row(4g + i, half) is bit 8g + i of
          // the lane's shifted word), sign-extended, selects its score or
          // -inf.  The threshold is at least -FLT_MAX, so a row passes it
          // only if it matches and scores at least the threshold, and the
          // candidate step runs only when some row of the wavefront does.
          const uint32_t mrow = m32 >> (4 * half);
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const uint32_t sel = (uint32_t)__builtin_amdgcn_sbfe(
                (int)mrow, 8 * (v >> 2) + (v & 3), 1);
            acc[v] = __uint_as_float((__float_as_uint(acc[v]) & sel) | (0xFF800000u & ~sel));
          }
          // best of each group of four rows (elements 4g .. 4g + 3)
          float gm[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            gm[g] = -INFINITY;
#pragma unroll
            for (int i = 0; i < 4; ++i) gm[g] = fmaxf(gm[g], acc[4 * g + i]);
          }
          float mx = -INFINITY;
#pragma unroll
          for (int g = 0; g < 4; ++g) mx = fmaxf(mx, gm[g]);
          const f32x16& s = acc;
          const float th = fmaxf(thr[b], -FLT_MAX);
          if (__ballot(mx >= th)) {
            {
              // wave-wide compaction: the v-th survivors of all lanes take
              // consecutive staging slots (this wavefront is the only writer
              // of its buffer, so the count needs no atomic); groups of four
              // rows with no survivor in any lane are passed over at once
              const uint32_t q = qi[b];
              const int jj = slot_j(b);
              const uint32_t room = (uint32_t)SR - (shead - tail0);
              uint32_t base = 0;
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                if (!__ballot(gm[g] >= th)) continue;
#pragma unroll
              for (int v = 4 * g; v < 4 * g + 4; ++v) {
                const bool on = s[v] >= th;
                const uint64_t bal = __ballot(on);
                if (bal == 0ull) continue;
                const uint32_t idx = base + __builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                base += (uint32_t)__popcll(bal);
                if (on) {
                  const uint64_t slot = (tile0 + u) * kTile + acc_row(v, half);
                  const uint32_t k32 = fkey(s[v]);
                  // the id (for the tie order) is looked up by the selection
                  const unsigned long long key =
                      ((unsigned long long)k32 << 32) | (unsigned long long)slot;
                  if (idx < room) {
                    s_sk[wave_s()][(shead + idx) % SR] = key;
                    s_sq[wave_s()][(shead + idx) % SR] = (uint8_t)jj;
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
              shead += base < room ? base : room;
            }
          }
        }
      }
      if (lane == 0) {
        lds_put(&s_shead[wave_s()], shead);
        lds_put(&s_done[wave_s()], sq + 1u);
      }
    }
    seq0 += n_s;
    if (lane == 0) lds_put(&s_fin[wave_s()], item_no);
    ++item_no;
    wg_barrier();                                     // item end
  }
}

// (dtype, padded dim, query blocks per wavefront, wavefronts per workgroup)
#define FR_SCAN_CASES(X) \
  X(kF32, 64, 1, 4) X(kF32, 128, 1, 4) X(kF32, 192, 1, 4) X(kF32, 256, 1, 4) \
  X(kBF16, 64, 2, 4) X(kF32, 64, 2, 4) X(kF32, 128, 2, 4) X(kBF16, 128, 2, 4) \
  X(kFP8, 256, 2, 4) \
  X(kBF16, 64, 1, 4) X(kBF16, 128, 1, 4) X(kBF16, 192, 1, 4) X(kBF16, 256, 1, 4) \
  X(kFP8, 64, 1, 4) X(kFP8, 64, 2, 4) X(kFP8, 128, 1, 4) X(kFP8, 128, 2, 4) \
  X(kFP8, 192, 1, 4) X(kFP8, 256, 1, 4) \
  X(kF32, 128, 1, 8) X(kBF16, 128, 1, 8) X(kFP8, 128, 1, 8)

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
  FR_REQUIRE(a.work);
  FR_REQUIRE(a.mw);
  if (dt == kFP8) {
    FR_REQUIRE(a.xscale);
    FR_REQUIRE(a.qscale);
  }
  if (a.tpi < 4 || a.tpi % 4 || n_wg < 1) return hipErrorInvalidValue;
  // the loader copies whole query tiles (128 or 256 positions) of mask words
  if (a.ppad < 256u || a.ppad % 256u) return hipErrorInvalidValue;
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

// Sort of n unique keys, descending, by rank: key i goes to position =
// the number of keys greater than it, found with n broadcast LDS reads per
// key.  For the short lists of the selections (n <= kRankSortMax) this is
// a few thousand cycles where the bitonic network's barrier stages take
// several times more.  Positions >= keep are dropped; val (optional)
// travels with its key; the destination must not overlap the source.
constexpr int kRankSortMax = 512;
__device__ void rank_sort_desc(const unsigned long long* key, const uint32_t* val, int n,
                               unsigned long long* dkey, uint32_t* dval, int keep) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const unsigned long long ki = key[i];
    int r = 0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) r += key[j] > ki ? 1 : 0;
    if (r < keep) {
      dkey[r] = ki;
      if (val) dval[r] = val[i];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// First pass only: the query could not be answered from this pass (why 1:
// its candidates overflowed the buffer; why 2: its speculative starting
// threshold proved above the K'-th best).  Set it up for the second pass
// and append it to that pass's list.  Called by the whole workgroup.
// Fine bucket (coarse * 16 + fine) where the count from the top of a query's
// histogram (kNBC coarse counters, then 16 fine ones per coarse bucket) first
// reaches kp; -1 when the histogram holds fewer.  Where the coarse and fine
// counts disagree, the coarse bucket's lowest fine bucket (the safe side).
__device__ int hist_cut(const uint32_t* h, uint32_t kp) {
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
    if (bstar < 0) bstar = c * 16;
  }
  return bstar;
}

// The query's histogram copied to LDS by the whole block (one round of
// loads instead of a serial chain of them in one thread).
__device__ void load_hist(const SelectArgs& a, uint32_t q, uint32_t* s_h) {
  const uint32_t* h = a.hist + (uint64_t)q * kHist;
  for (int i = threadIdx.x; i < kHist; i += blockDim.x) s_h[i] = h[i];
  __syncthreads();
}

__device__ void select_rerun(const SelectArgs& a, uint32_t q, uint32_t why, uint32_t* s_h) {
  uint32_t* h = a.hist + (uint64_t)q * kHist;
  if (why != 2u) load_hist(a, q, s_h);
  if (threadIdx.x == 0) {
    float lo, hi;
    if (why == 2u) {
      // every match at or above the speculative start was seen (the
      // largest is smax), the rest lie below it: scan again from the safe
      // start
      hi = fmaxf(key2f(a.smax[q]), key2f(a.tau[q]));
      a.tau[q] = a.tsafe[q];
      lo = key2f(a.tsafe[q]);
      if (!isfinite(lo)) lo = -(a.qnorm[q] * __uint_as_float(*a.norm_max) * 1.0001f);
    } else {
      // raise the threshold from the complete first-pass histogram (the
      // scan's own refreshes may have seen only part of it): same bucket
      // rule and one-bucket margin as the scan's refresh
      const uint32_t kp = a.kp[q];
      const float lo0 = a.hlo[q], iw0 = a.hinvw[q];
      const int bstar = hist_cut(s_h, kp);
      if (kp && bstar >= 2 && iw0 > 0.f) {
        const uint32_t nk = fkey(lo0 + (float)(bstar - 1) / iw0);
        if (nk > a.tau[q]) a.tau[q] = nk;
      }
      lo = key2f(a.tau[q]);
      hi = key2f(a.smax[q]);
    }
    a.tsafe[q] = 0u;
    const float span = (hi - lo) * 1.0001f;
    const bool ok = span > 0.f && isfinite(span) && isfinite(lo);
    a.hlo[q] = ok ? lo : 0.f;
    a.hinvw[q] = ok ? (float)kNBF / span : 0.f;
    a.cnt[q] = 0u;
    a.smax[q] = 0u;
    a.sel_cnt[q] = 0u;
    const uint32_t p = atomicAdd(a.n_list2, 1u);
    a.qlist2[p] = q;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHist; i += blockDim.x) h[i] = 0u;
}

// Exact top-kp of one query's candidates (those at or above the final
// threshold), sorted by key descending = (score desc, id asc).
__global__ __launch_bounds__(256) void k_select(SelectArgs a) {
  __shared__ unsigned long long s_key[kSelCap];
  __shared__ uint32_t s_slot[kSelCap];
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_h[kHist];
  __shared__ uint32_t s_n, s_digit, s_rank;
  const uint32_t pos = blockIdx.x;
  // the first pass's scan is over: its work counters serve the second one
  if (!a.final_pass && blockIdx.x == 0 && threadIdx.x < kXcds) a.work[threadIdx.x] = 0u;
  if (pos >= *a.n_list) return;
  const uint32_t q = a.qlist[pos];
  const uint32_t kp = a.kp[q];
  const uint32_t c = a.cnt[q];
  if (c > a.cap) {
    // Candidates were dropped: scan the query again, or, if this was the
    // second pass, mark it failed (count 0xFFFFFFFF, no ids).
    if (!a.final_pass) {
      select_rerun(a, q, 1u, s_h);
      return;
    }
    if (threadIdx.x == 0) {
      a.ovf[q] = 1u;
      a.sel_cnt[q] = 0u;
    }
    if (a.write_out) {
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
  if (!a.final_pass && a.tsafe[q] != 0u && (unsigned long long)c < min((unsigned long long)kp, a.nmatch[q])) {
    // The speculative starting threshold was above the K'-th best match
    // (fewer candidates than min(K', matches) reached it): scan again from
    // the safe one.
    select_rerun(a, q, 2u, s_h);
    return;
  }
  // Cut before sorting: the query's histogram counts exactly this pass's
  // candidates, so the lower edge of the bucket below the one where the
  // count from the top reaches kp is at most the kp-th best candidate
  // (the same bucket rule as the scan's threshold refresh); candidates below
  // max(tau, that edge) cannot be selected.
  __shared__ uint32_t s_tau;
  load_hist(a, q, s_h);
  if (threadIdx.x == 0) {
    uint32_t t = a.tau[q];
    const float lo0 = a.hlo[q], iw0 = a.hinvw[q];
    const int bstar = hist_cut(s_h, kp);
    if (kp && bstar >= 2 && iw0 > 0.f) t = max(t, fkey(lo0 + (float)(bstar - 1) / iw0));
    s_tau = t;
  }
  __syncthreads();
  const uint32_t tau = s_tau;
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
  const uint32_t out = min(kp, m);
  unsigned long long* skey = s_key;
  uint32_t* sslot = s_slot;
  static_assert(kSelCap >= 2 * kRankSortMax, "rank sort destination");
  if (m <= (uint32_t)kRankSortMax) {
    skey = s_key + kRankSortMax;
    sslot = s_slot + kRankSortMax;
    rank_sort_desc(s_key, s_slot, (int)m, skey, sslot, (int)out);
  } else {
    const int n2 = pow2_at_least((int)m);
    for (int i = (int)m + threadIdx.x; i < n2; i += blockDim.x) {
      s_key[i] = 0ull;
      s_slot[i] = 0xFFFFFFFFu;
    }
    __syncthreads();
    bitonic_desc(s_key, s_slot, n2);
  }
  for (uint32_t r = threadIdx.x; r < out; r += blockDim.x) {
    a.sel_key[(uint64_t)q * a.rmax + r] = skey[r];
    a.sel_slot[(uint64_t)q * a.rmax + r] = sslot[r];
  }
  if (threadIdx.x == 0) a.sel_cnt[q] = out;
  if (a.write_out) {
    const uint32_t kq = min(a.k[q], out);
    for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
      const bool ok = r < kq;
      const unsigned long long k = ok ? skey[r] : 0ull;
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
  FR_REQUIRE(a.tsafe);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.hist);
  FR_REQUIRE(a.smax);
  FR_REQUIRE(a.hlo);
  FR_REQUIRE(a.hinvw);
  FR_REQUIRE(a.qlist2);
  FR_REQUIRE(a.n_list2);
  FR_REQUIRE(a.work);
  FR_REQUIRE(a.qnorm);
  FR_REQUIRE(a.norm_max);
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
  __shared__ unsigned long long s_sur[kMaxR];   // keys that survive the bucket cut
  __shared__ uint32_t s_cnt[256];
  __shared__ uint32_t s_kmin, s_kmax, s_cut, s_n;
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
  // wavefront `wave` rescores rows [rb, re): their slots and ids are read
  // 64 at a time (one per lane), then 16 rows are gathered at once
  const uint32_t per = (m + 3u) / 4u;
  const uint32_t rb = min(m, (uint32_t)wave * per), re = min(m, rb + per);
  for (uint32_t c0 = rb; c0 < re; c0 += 64u) {
    const uint32_t nr = min(64u, re - c0);
    const uint32_t my_slot = (uint32_t)lane < nr ? ss[c0 + lane] : 0u;
    const uint32_t my_id = (uint32_t)lane < nr ? (uint32_t)sk[c0 + lane] : 0u;
    for (uint32_t j0 = 0; j0 < nr; j0 += 16u) {
      float4 xv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint32_t j = j0 + (uint32_t)u;
        const uint32_t slot = (uint32_t)__shfl((int)my_slot, (int)(j & 63u));
        xv[u] = (on && j < nr) ? *((const float4*)(a.master + (uint64_t)slot * a.dpad) + lane)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        float p = xv[u].x * qv.x;
        p = fmaf(xv[u].y, qv.y, p);
        p = fmaf(xv[u].z, qv.z, p);
        p = fmaf(xv[u].w, qv.w, p);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) p += __shfl_xor(p, off);
        const uint32_t j = j0 + (uint32_t)u;
        const uint32_t id = (uint32_t)__shfl((int)my_id, (int)(j & 63u));
        if (lane == 0 && j < nr)
          s_key[c0 + j] = ((unsigned long long)fkey(p) << 32) | (unsigned long long)id;
      }
    }
  }
  __syncthreads();
  const uint32_t kq = min(a.k[q], m);
  // Only the best kq keys are output: with many rows, keep the 256-bucket
  // buckets (over the score keys' integer range, so bucket order is key
  // order exactly) from the one holding the kq-th key upwards, and sort
  // those survivors only.
  unsigned long long* srt = s_key;
  uint32_t n = m;
  if (m > 512u && kq) {
    if (threadIdx.x == 0) {
      s_kmin = 0xFFFFFFFFu;
      s_kmax = 0u;
      s_n = 0u;
    }
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_cnt[i] = 0u;
    __syncthreads();
    uint32_t lmin = 0xFFFFFFFFu, lmax = 0u;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      const uint32_t hk = (uint32_t)(s_key[i] >> 32);
      lmin = min(lmin, hk);
      lmax = max(lmax, hk);
    }
    atomicMin(&s_kmin, lmin);
    atomicMax(&s_kmax, lmax);
    __syncthreads();
    const uint32_t kmin = s_kmin;
    const uint64_t span = (uint64_t)(s_kmax - kmin) + 1ull;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      const uint32_t hk = (uint32_t)(s_key[i] >> 32);
      atomicAdd(&s_cnt[(uint32_t)(((uint64_t)(hk - kmin) << 8) / span)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t cum = 0u;
      int b = 255;
      for (; b > 0; --b) {
        cum += s_cnt[b];
        if (cum >= kq) break;
      }
      // lower edge of bucket b: the least key whose bucket is b
      s_cut = kmin + (uint32_t)(((uint64_t)b * span + 255ull) >> 8);
    }
    __syncthreads();
    const uint32_t cut = s_cut;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      const unsigned long long k = s_key[i];
      if ((uint32_t)(k >> 32) >= cut) s_sur[atomicAdd(&s_n, 1u)] = k;
    }
    __syncthreads();
    srt = s_sur;
    n = s_n;
  }
  if (n <= (uint32_t)kRankSortMax) {
    unsigned long long* dst = srt == s_key ? s_sur : s_key;   // the other buffer
    rank_sort_desc(srt, nullptr, (int)n, dst, nullptr, (int)kq);
    srt = dst;
  } else {
    const int n2 = pow2_at_least((int)n);
    for (int i = (int)n + threadIdx.x; i < n2; i += blockDim.x) srt[i] = 0ull;
    __syncthreads();
    bitonic_desc(srt, nullptr, n2);
  }
  for (uint32_t r = threadIdx.x; r < a.k_max; r += blockDim.x) {
    const bool ok = r < kq;
    const unsigned long long k = ok ? srt[r] : 0ull;
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
