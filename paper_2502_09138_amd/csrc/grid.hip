// K1: per-(sector,row) grid -- step C1 of the tracker definition.
//
// One workgroup per pack of consecutive rows (one row if it has more than
// kPackHits hits, else as many rows as fit kPackHits hits and kPackRows rows):
// the rows of a pack are contiguous in the input and in the output, so they
// are sorted together on the key (row, bin), whose exclusive scan gives every
// row's sorted positions at once.  Bins come from the exact float32 rule; the
// order in a row is a stable counting sort by (bin, input id):
//   1. bin every hit, LDS-atomic histogram (the returned slot is arbitrary),
//   2. exclusive scan of the histogram -> bin starts,
//   3. scatter local ids into their bins at the arbitrary slot,
//   4. each position ranks its id among the (few) ids of its own bin, which
//      restores input order inside the bin without a global sort.
// Coordinates are checked for NaN/Inf and |.| > TPC_MAX_COORD on the way.
#include <algorithm>

#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kLdsRowCap = 4096;        // rows up to this many hits run from LDS

// cnt[nb+1] (32-bit: bin counts, then bin starts); key[n], slot[n], tmp[n] as
// 16-bit values (bin index < nb <= 65535, rank inside a bin and local id < n <=
// 65535), which halves the LDS a row needs and so doubles the rows resident
// per CU.
struct RowArrays {
  uint32_t* cnt;
  uint16_t* key;
  uint16_t* slot;
  uint16_t* tmp;
};

__device__ void grid_row(const DevPtrs& d, uint32_t sr, const RowArrays& A, uint32_t* wsum) {
  const int grid_k = d.grid_k;
  const uint32_t R = d.R;
  const uint32_t s = sr / R, row = sr % R;
  const uint32_t a = d.row_off[sr];
  const uint32_t n = d.row_off[sr + 1] - a;
  const RowConst rc = d.rows[row];
  const SectorConst sc = d.secs[s];
  int ny, nz;
  grid_dims(n, grid_k, rc.ly, sc.lz, ny, nz);
  const uint32_t nb = (uint32_t)(ny * nz);
  if (threadIdx.x == 0) {
    d.row_dims[sr] = (uint32_t)ny | ((uint32_t)nz << 16);
    d.row_meta[sr] = make_uint2(bin_base(d, sr), (uint32_t)ny | ((uint32_t)nz << 16));
  }
  for (uint32_t b = threadIdx.x; b <= nb; b += blockDim.x) A.cnt[b] = 0;
  __syncthreads();
  bool bad = false;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const float yv = d.y[a + j], zv = d.z[a + j];
    bad |= !(fabsf(yv) <= kMaxCoord) || !(fabsf(zv) <= kMaxCoord);
    const int iy = bin1(yv, rc.y_lo, rc.inv_wy, ny);
    const int iz = bin1(zv, sc.z_lo, sc.inv_wz, nz);
    const uint32_t b = (uint32_t)(iz * ny + iy);
    A.key[j] = (uint16_t)b;
    A.slot[j] = (uint16_t)atomicAdd(&A.cnt[b], 1u);
  }
  if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&d.hdr->error_flags, 1u);
  __syncthreads();
  block_scan_array(A.cnt, nb, wsum);
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) A.tmp[A.cnt[A.key[j]] + A.slot[j]] = j;
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < n; p += blockDim.x) {
    const uint32_t j = A.tmp[p];
    const uint32_t b = A.key[j];
    const uint32_t b0 = A.cnt[b], b1 = A.cnt[b + 1];
    uint32_t rank = 0;
    for (uint32_t q = b0; q < b1; ++q) rank += (uint32_t)A.tmp[q] < j;
    const uint32_t out = a + b0 + rank;
    d.sid[out] = a + j;
    d.syz[out] = make_float2(d.y[a + j], d.z[a + j]);
  }
  __syncthreads();
  // row-local bin starts -> global sorted positions (in place when cnt is the bin_start row itself)
  const uint32_t base = bin_base(d, sr);
  for (uint32_t b = threadIdx.x; b <= nb; b += blockDim.x) d.bin_start[base + b] = a + A.cnt[b];
  // the row's entries of the neighbour finder's tile -> row map
  for (uint32_t t = d.tile_off[sr] + threadIdx.x; t < d.tile_off[sr + 1]; t += blockDim.x) d.tile_sr[t] = sr;
}

// LDS of a pack of up to cap hits: cnt_words 32-bit bin counts (at most
// max(1, n_p / K) bins per row, so cap / K + kPackRows, plus the end entry,
// rounded to an even count so the 16-bit arrays start 4-byte aligned), then
// three 16-bit arrays of cap entries.
__host__ __device__ inline uint32_t cnt_words(uint32_t cap, int k) {
  return ((cap / (uint32_t)k + kPackRows + 1) + 1u) & ~1u;
}

__global__ void __launch_bounds__(kThreads) k_grid_lds(DevPtrs d, uint32_t cap) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t wsum[kThreads / kWave];
  // per row of the pack: local start (lst[P] = the pack's hits), first bin (boff[P] = its bins), bin rule
  __shared__ uint32_t lst[kPackRows + 1], boff[kPackRows + 1];
  __shared__ float ylo[kPackRows], iwy[kPackRows], zlo[kPackRows], iwz[kPackRows];
  __shared__ int nyv[kPackRows], nzv[kPackRows];
  const uint32_t sr0 = d.pack_first[blockIdx.x], sr1 = d.pack_first[blockIdx.x + 1], P = sr1 - sr0;
  const uint32_t a0 = d.row_off[sr0];
  const uint32_t n = d.row_off[sr1] - a0;
  if (n > cap) return;            // a single row beyond the LDS capacity: k_grid_global
  const uint32_t R = d.R;
  if (threadIdx.x < P) {
    const uint32_t p = threadIdx.x, sr = sr0 + p;
    const uint32_t np = d.row_off[sr + 1] - d.row_off[sr];
    const RowConst rc = d.rows[sr % R];
    const SectorConst sc = d.secs[sr / R];
    int ny, nz;
    grid_dims(np, d.grid_k, rc.ly, sc.lz, ny, nz);
    d.row_dims[sr] = (uint32_t)ny | ((uint32_t)nz << 16);
    d.row_meta[sr] = make_uint2(bin_base(d, sr), (uint32_t)ny | ((uint32_t)nz << 16));
    lst[p] = d.row_off[sr] - a0;
    boff[p] = (uint32_t)(ny * nz);   // bins of row p, turned into offsets below
    ylo[p] = rc.y_lo;
    iwy[p] = rc.inv_wy;
    zlo[p] = sc.z_lo;
    iwz[p] = sc.inv_wz;
    nyv[p] = ny;
    nzv[p] = nz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t o = 0;
    for (uint32_t p = 0; p < P; ++p) {
      const uint32_t nb = boff[p];
      boff[p] = o;
      o += nb;
    }
    boff[P] = o;
    lst[P] = n;
  }
  __syncthreads();
  const uint32_t NB = boff[P];
  uint16_t* key = reinterpret_cast<uint16_t*>(lds + cnt_words(cap, d.grid_k));
  uint16_t* slot = key + cap;
  uint16_t* tmp = key + 2 * cap;
  uint32_t* cnt = lds;
  for (uint32_t b = threadIdx.x; b <= NB; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  bool bad = false;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    uint32_t lo = 0, hi = P;   // the row of hit j: last p with lst[p] <= j (empty rows share their start)
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (lst[mid] <= j) lo = mid;
      else hi = mid;
    }
    const float yv = d.y[a0 + j], zv = d.z[a0 + j];
    bad |= !(fabsf(yv) <= kMaxCoord) || !(fabsf(zv) <= kMaxCoord);
    const int ny = nyv[lo];
    const int iy = bin1(yv, ylo[lo], iwy[lo], ny);
    const int iz = bin1(zv, zlo[lo], iwz[lo], nzv[lo]);
    const uint32_t b = boff[lo] + (uint32_t)(iz * ny + iy);
    key[j] = (uint16_t)b;
    slot[j] = (uint16_t)atomicAdd(&cnt[b], 1u);
  }
  if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&d.hdr->error_flags, 1u);
  __syncthreads();
  block_scan_array(cnt, NB, wsum);
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) tmp[cnt[key[j]] + slot[j]] = (uint16_t)j;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
    const uint32_t j = tmp[q];
    const uint32_t b = key[j];
    const uint32_t b0 = cnt[b], b1 = cnt[b + 1];
    uint32_t rank = 0;
    for (uint32_t u = b0; u < b1; ++u) rank += (uint32_t)tmp[u] < j;
    const uint32_t out = a0 + b0 + rank;
    d.sid[out] = a0 + j;
    d.syz[out] = make_float2(d.y[a0 + j], d.z[a0 + j]);
  }
  // bin starts (row p's end entry is row p + 1's first start) and the K2 tile -> row map
  for (uint32_t p = 0; p < P; ++p) {
    const uint32_t sr = sr0 + p, base = bin_base(d, sr), b0 = boff[p], nb = boff[p + 1] - b0;
    for (uint32_t b = threadIdx.x; b <= nb; b += blockDim.x) d.bin_start[base + b] = a0 + cnt[b0 + b];
    for (uint32_t t = d.tile_off[sr] + threadIdx.x; t < d.tile_off[sr + 1]; t += blockDim.x) d.tile_sr[t] = sr;
  }
}

// Rows larger than the LDS capacity: the same steps with the arrays in global
// memory.  The counts use the row's own bin_start slots (n + 2 >= nBins + 1);
// key/slot/order use the row's range of the C2/C3 link arrays, which are
// written only later.
__global__ void __launch_bounds__(kThreads) k_grid_global(DevPtrs d, uint32_t cap) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t sr = blockIdx.x;
  const uint32_t a = d.row_off[sr];
  const uint32_t n = d.row_off[sr + 1] - a;
  if (n <= cap) return;
  RowArrays A{d.bin_start + bin_base(d, sr), reinterpret_cast<uint16_t*>(d.up0 + a),
              reinterpret_cast<uint16_t*>(d.down0 + a), reinterpret_cast<uint16_t*>(d.up1 + a)};
  grid_row(d, sr, A, wsum);
}

}  // namespace

void launch_grid(const DevPtrs& d, uint32_t max_row_hits, uint32_t max_pack_hits, hipStream_t s) {
  if (d.SR == 0) return;
  // every pack of several rows has at most kPackHits <= kLdsRowCap hits, so only single rows exceed cap
  const uint32_t cap = std::max<uint32_t>(1u, max_pack_hits < kLdsRowCap ? max_pack_hits : kLdsRowCap);
  const size_t lds = (size_t)cnt_words(cap, d.grid_k) * sizeof(uint32_t) + (size_t)3 * cap * sizeof(uint16_t);
  hipLaunchKernelGGL(k_grid_lds, dim3(d.n_packs), dim3(kThreads), lds, s, d, cap);
  if (max_row_hits > kLdsRowCap) hipLaunchKernelGGL(k_grid_global, dim3(d.SR), dim3(kThreads), 0, s, d, cap);
}

}  // namespace tpc
