// Selectivity-adaptive routing for gfx950 (appendix "Message Passing between
// Layers" and "EBR": a stage hands the next one the list of rows that passed
// it, and EBR scores only those rows, which pays when few rows pass).  A
// query whose predicate matches few documents skips the dense scan: its
// matching slots are listed from its mask words and each listed row is
// scored by one wavefront in FP32; the exact selection then takes its top K
// as for any other query.  The scan keeps the remaining queries, so the
// matrix-core work shrinks by whole query blocks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {

// ------------------------------------------------------------ routing
// One workgroup of 1024 threads: a stable partition of queries 0..n-1 into
// the scan's list and the sparse list (ballot counts per wavefront, their
// prefix in LDS).
__global__ __launch_bounds__(1024) void k_route(RouteArgs a) {
  __shared__ uint32_t s_d[16], s_s[16];
  __shared__ uint32_t s_nd, s_ns;
  const uint32_t n = min(*a.n_dev, a.max_q);
  const int lane = threadIdx.x & 63;
  const uint32_t wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    s_nd = 0u;
    s_ns = 0u;
  }
  __syncthreads();
  for (uint32_t base = 0; base < n; base += 1024u) {
    const uint32_t q = base + threadIdx.x;
    const bool ok = q < n;
    bool sp = false;
    if (ok) {
      unsigned long long lim = a.limit;
      if (a.cap_by_kp) lim = min(lim, (unsigned long long)a.kp[q]);
      sp = a.nmatch[q] <= lim;
    }
    const unsigned long long bs = __ballot(ok && sp), bd = __ballot(ok && !sp);
    if (lane == 0) {
      s_s[wv] = (uint32_t)__popcll(bs);
      s_d[wv] = (uint32_t)__popcll(bd);
    }
    __syncthreads();
    uint32_t os = s_ns, od = s_nd;
    for (uint32_t i = 0; i < wv; ++i) {
      os += s_s[i];
      od += s_d[i];
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    if (ok) {
      if (sp) a.slist[os + (uint32_t)__popcll(bs & below)] = q;
      else a.qlist[od + (uint32_t)__popcll(bd & below)] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 0; i < 16; ++i) {
        s_ns += s_s[i];
        s_nd += s_d[i];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *a.n_list = s_nd;
    *a.n_slist = s_ns;
  }
}
hipError_t launch_route(const RouteArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.nmatch);
  FR_REQUIRE(a.qlist);
  FR_REQUIRE(a.n_list);
  FR_REQUIRE(a.slist);
  FR_REQUIRE(a.n_slist);
  if (a.cap_by_kp) FR_REQUIRE(a.kp);
  hipLaunchKernelGGL(k_route, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------- row listing
// Blocks of 256 threads over (group range, sparse query): each thread holds
// one mask word, a wavefront prefix sum of the words' bit counts gives each
// thread its place after one counter update per wavefront, and the thread
// writes its word's slots in order.
__global__ __launch_bounds__(256) void k_sparse_rows(SparseRowsArgs a) {
  const uint32_t n_y = min(*a.n_slist, a.max_q);
  const int lane = threadIdx.x & 63;
  const uint32_t w0 = blockIdx.x * a.gpb * (uint32_t)kWords;
  const uint32_t w1 = min((blockIdx.x + 1u) * a.gpb, a.n_groups) * (uint32_t)kWords;
  for (uint32_t y = blockIdx.y; y < n_y; y += gridDim.y) {
  const uint32_t q = a.slist[y];
  uint32_t* out = a.rows + (uint64_t)q * a.cap;
  for (uint32_t base = w0; base < w1; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const uint64_t m = i < w1 ? a.mw[(uint64_t)i * a.ppad + q] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    uint32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)x, off);
      if (lane >= off) x += v;
    }
    const uint32_t total = (uint32_t)__shfl((int)x, 63);
    uint32_t pos = 0;
    if (lane == 0 && total) pos = atomicAdd(a.cnt + q, total);
    pos = (uint32_t)__shfl((int)pos, 0) + x - c;
    uint64_t mm = m;
    while (mm) {
      const uint32_t b = (uint32_t)(__ffsll((long long)mm) - 1);
      mm &= mm - 1ull;
      if (pos < a.cap) out[pos] = i * 64u + b;
      ++pos;
    }
  }
  }
}
hipError_t launch_sparse_rows(const SparseRowsArgs& a, hipStream_t s) {
  FR_REQUIRE(a.slist);
  FR_REQUIRE(a.n_slist);
  FR_REQUIRE(a.mw);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.rows);
  if (!a.max_q || !a.n_groups) return hipSuccess;
  if (a.gpb < 1 || a.ppad < a.max_q) return hipErrorInvalidValue;
  // the sparse list's length is known on the device only: a few blocks per
  // group range loop over it
  hipLaunchKernelGGL(k_sparse_rows, dim3((a.n_groups + a.gpb - 1) / a.gpb, min(a.max_q, 32u)),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------- row scores
// Element e of a slot's row in the FP32 embedding tiles: the tile of 32
// rows, the row's half, its 16-byte chunk and the element in the chunk.
__device__ __forceinline__ float tile_elem(const uint8_t* tiles, uint64_t slot, uint32_t dpad,
                                           uint32_t e) {
  const uint32_t hd = dpad / 2u, h = e / hd, p = e % hd;
  const uint8_t* tile = tiles + (slot / kTile) * ((uint64_t)kTile * dpad * 4u);
  const uint32_t r = (uint32_t)(slot % kTile);
  return *(const float*)(tile + ((size_t)((p / 4u) * 64u + h * 32u + r) * 16u) + (p % 4u) * 4u);
}

// One wavefront per listed row: lane l multiplies coordinates l, l+64, ...
// (FP32 FMA), then a fixed butterfly sums the lanes.  Blocks of 4
// wavefronts cover 64 rows of one query (grid.y = query or list position).
__global__ __launch_bounds__(256) void k_row_dots(RowDotArgs a) {
  const uint32_t n_y = min(a.qlist ? *a.n_list : *a.n_dev, a.max_q);
  const int lane = threadIdx.x & 63;
  for (uint32_t y = blockIdx.y; y < n_y; y += gridDim.y) {
  const uint32_t q = a.qlist ? a.qlist[y] : y;
  const uint32_t c = a.cnt[q];
  if (c > a.stride) continue;   // failed query
  const float* qr = a.qrows + (uint64_t)q * a.q_ld;
  const uint32_t* rl = a.rows + (uint64_t)q * a.stride;
  const uint32_t i0 = blockIdx.x * 64u + (threadIdx.x >> 6) * 16u;
  const float hlo = a.hist ? a.hlo[q] : 0.f, hiw = a.hist ? a.hinvw[q] : 0.f;
  for (uint32_t i = i0; i < min(i0 + 16u, c); ++i) {
    const uint32_t slot = rl[i];
    float p = 0.f;
    if (a.master) {
      const float* xr = a.master + (uint64_t)slot * a.dpad;
      for (uint32_t d = (uint32_t)lane; d < a.dim; d += 64u) p = fmaf(xr[d], qr[d], p);
    } else {
      for (uint32_t d = (uint32_t)lane; d < a.dim; d += 64u)
        p = fmaf(tile_elem(a.tiles, slot, a.dpad, d), qr[d], p);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off);
    if (lane == 0) {
      a.key[(uint64_t)q * a.key_stride + i] = ((unsigned long long)fkey(p) << 32) | slot;
      if (a.hist) {
        const float fb = (p - hlo) * hiw;
        const int bk = fb >= (float)(kNBF - 1) ? kNBF - 1 : (fb > 0.f ? (int)fb : 0);
        uint32_t* hq = a.hist + (uint64_t)q * kHist;
        atomicAdd(hq + kNBC + bk, 1u);
        atomicAdd(hq + (bk >> 4), 1u);
      }
    }
  }
  }
}
hipError_t launch_row_dots(const RowDotArgs& a, hipStream_t s) {
  FR_REQUIRE(a.n_dev);
  FR_REQUIRE(a.cnt);
  FR_REQUIRE(a.rows);
  FR_REQUIRE(a.qrows);
  FR_REQUIRE(a.key);
  if (!a.master) FR_REQUIRE(a.tiles);
  if (a.qlist) FR_REQUIRE(a.n_list);
  if (!a.max_q || !a.max_cnt) return hipSuccess;
  if (a.dim > a.dpad || a.dpad % 64u || a.q_ld < a.dim || a.max_cnt > a.stride ||
      a.key_stride < a.stride)
    return hipErrorInvalidValue;
  if (a.hist) {
    FR_REQUIRE(a.hlo);
    FR_REQUIRE(a.hinvw);
  }
  hipLaunchKernelGGL(k_row_dots, dim3((a.max_cnt + 63) / 64, min(a.max_q, 64u)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace fr
