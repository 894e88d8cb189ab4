// fn_knn.h -- Parents(T, x, M) of Algorithm 1: brute-force k nearest tree
// nodes by Euclidean distance in the 14-D state space (Sec. IV-E).
//
// Stage 1 (knn_scan): one wavefront per (4 queries, node chunk); lanes run
// over the chunk's nodes with coalesced loads of the SoA tree rows, every
// screening distance costs 14 FMAs, and each query keeps its chunk's K1
// smallest FP32 keys (d^2, index), K1 >= k + 4 (knn_k1), sorted over
// lanes 0..K1-1.
// Stage 2 (knn_merge): one wavefront per query merges the chunk lists.  The
// FP32 k-th key bounds a band that provably holds the exact top-k; every
// list entry in the band is re-ranked with the FP64 distance summed in the
// reference order (c = 0..13, separately rounded products and sums).  When
// a chunk's last (K1-th) entry also falls in the band, that chunk may hold
// more in-band nodes than its list, and the query is rescanned exactly in
// FP64; the spare entries make this rare.
#pragma once

#include <hip/hip_runtime.h>

#include "fn_ctx.h"

namespace fn {

constexpr int KNN_TARGET_WAVES = 4096;
// Largest tree leading dimension: the scan addresses the 14 rows with 32-bit
// byte offsets (14 * ld * 4 < 2^31).
constexpr int64_t KNN_MAX_LD = (((int64_t)1 << 31) - 1) / (4 * FN_STATE) / 4 * 4;
constexpr float KNN_BAND = 1e-6f;  // slack for rounding the band itself
constexpr float KNN_EPS = 4e-6f;   // |d32 - d| <= KNN_EPS (|x| + |y|)^2 (twice the FP32 bound)

__device__ __forceinline__ bool key_less(float d, int i, float d2, int i2) {
  return d < d2 || (d == d2 && (unsigned)i < (unsigned)i2);
}

// lane r takes lane r-1's value (DPP wave shift; lane 0 gets 0)
__device__ __forceinline__ float wave_shr1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138,
                                                            0xf, 0xf, true));
}
__device__ __forceinline__ int wave_shr1(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

// Value of lane (lane ^ J) (J a power of two below 64): DPP quad
// permutations for 1 and 2, LDS swizzle (bit-mask mode, within 32 lanes)
// for 4..16, LDS permute for 32.
template <int J>
__device__ __forceinline__ int lane_xor(int v) {
  if constexpr (J == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
  else if constexpr (J == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, true);  // 2,3,0,1
  else if constexpr (J < 32) return __builtin_amdgcn_ds_swizzle(v, (J << 10) | 0x1f);
  else return __builtin_amdgcn_ds_bpermute((int)((threadIdx.x & 63) ^ 32) << 2, v);
}

// (d, i) as one unsigned 64-bit key ordered as key_less: the float's bits
// mapped to an order-preserving unsigned value, then the index (unsigned,
// so the -1 of a padding entry ranks last).
__device__ __forceinline__ uint64_t knn_key(float d, int i) {
  const uint32_t b = __float_as_uint(d + 0.f);  // -0 -> +0, as key_less treats them equal
  const uint32_t m = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)m << 32) | (uint32_t)i;
}
__device__ __forceinline__ float knn_key_d(uint64_t k) {
  const uint32_t m = (uint32_t)(k >> 32);
  return __uint_as_float((m & 0x80000000u) ? (m & 0x7fffffffu) : ~m);
}

// One compare-exchange stage (block size K, distance J) of the bitonic
// network over the 64 lanes' keys.
template <int K, int J>
__device__ __forceinline__ void bitonic_stage(uint64_t& key) {
  const int lane = threadIdx.x & 63;
  const uint64_t o = ((uint64_t)(uint32_t)lane_xor<J>((int)(key >> 32)) << 32) |
                     (uint32_t)lane_xor<J>((int)(uint32_t)key);
  // the lower lane of a pair keeps the smaller key in an ascending block of
  // size K, the larger one in a descending block
  const bool want_min = ((lane & J) == 0) == ((lane & K) == 0);
  key = (want_min ? o < key : key < o) ? o : key;
}

template <int K, int J>
__device__ __forceinline__ void bitonic_merge_steps(uint64_t& key) {
  bitonic_stage<K, J>(key);
  if constexpr (J > 1) bitonic_merge_steps<K, J / 2>(key);
}

// Sorts the 64 lanes' keys (d, i) ascending by key_less (bitonic network
// over 64-bit keys; equal keys stay put).
__device__ __forceinline__ void wave_sort64(float& d, int& i) {
  uint64_t key = knn_key(d, i);
  bitonic_merge_steps<2, 1>(key);
  bitonic_merge_steps<4, 2>(key);
  bitonic_merge_steps<8, 4>(key);
  bitonic_merge_steps<16, 8>(key);
  bitonic_merge_steps<32, 16>(key);
  bitonic_merge_steps<64, 32>(key);
  d = knn_key_d(key);
  i = (int)(uint32_t)key;
}

// LDS of one scan wavefront: per query, a buffer of candidate keys.
template <int QG>
struct KnnBuf {
  float d[QG][WAVE];
  int32_t i[QG][WAVE];
};

// One wavefront per (QG queries, node chunk).  Lanes run over 64 nodes at
// a time (coalesced loads of the SoA rows).  The FP32 screening distance is
// |x|^2 + |y|^2 - 2 x.y (14 FMAs per pair, |y|^2 shared by the QG queries);
// its absolute error is below 4e-6 (|x| + |y|)^2, a bound the merge carries
// into the band it re-ranks exactly.  Every query keeps its chunk's K1
// best keys (d^2, index) sorted over lanes 0..K1-1 with the K1-th as a
// wave-uniform threshold.  A node that beats the threshold is appended to
// the query's LDS buffer (ballot + lane rank); when the list and the buffer
// fill the 64 lanes they are sorted together and the list and threshold
// are renewed.  Nodes arrive in increasing index, so a node whose distance
// equals the threshold never beats it, and every node left out has a key
// above the chunk's final K1-th key: the list is the chunk's exact FP32
// top K1 by (d^2, index).
// Node tiles shared by the 4 wavefronts of a workgroup (tiled form): 256
// nodes x (14 coordinates, |y|^2), row stride 17 so that the 64 lanes of a
// wavefront reading 64 consecutive rows hit distinct banks.
constexpr int KNN_TILE = 256;
constexpr int KNN_TILE_LD = FN_STATE + 3;

// TILED = false: the wavefront loads its own node rows (several query groups
// of one workgroup may scan different chunks).  TILED = true: the workgroup's
// wavefronts all scan chunk ch, and each tile of 256 nodes is loaded once
// into LDS with |y|^2 (the same FMA chain as the untiled form, so the keys
// are bit-identical) for the 4 x QG queries; `active` = false for a
// wavefront past the last query group (it still loads and synchronises).
template <int K1, int QG, bool TILED = false>
__device__ void knn_scan_item(const float* __restrict__ tree, int64_t ld, int n_nodes,
                              const float* __restrict__ qs, int B, int grp, int ch, int n_split,
                              int chunk, float* __restrict__ out_d, int32_t* __restrict__ out_i,
                              float* __restrict__ out_y2, KnnBuf<QG>* buf, bool active = true,
                              float* tile = nullptr) {
  constexpr int CAP = WAVE - K1;  // buffer entries that fit beside the list
  const int lane = threadIdx.x & 63;
  float xm2[QG][FN_STATE], xx[QG];
#pragma unroll
  for (int q = 0; q < QG; ++q) {
    const int b = min(grp * QG + q, B - 1);
    float s2 = 0.f;
#pragma unroll
    for (int c = 0; c < FN_STATE; ++c) {
      const float v = qs[(size_t)b * FN_STATE + c];
      xm2[q][c] = -2.f * v;
      s2 = fmaf(v, v, s2);
    }
    xx[q] = s2;
  }
  float Ld[QG];
  int Li[QG];
  float th_d[QG];
  int nb[QG];
#pragma unroll
  for (int q = 0; q < QG; ++q) {
    Ld[q] = INFINITY;
    Li[q] = -1;
    th_d[q] = INFINITY;
    nb[q] = 0;
  }
  // list + buffer of query q sorted together; list and threshold renewed
  auto merge = [&](int q) {
    __builtin_amdgcn_wave_barrier();
    const int t = lane - K1;
    float d = lane < K1 ? Ld[q] : (t < nb[q] ? buf->d[q][t] : INFINITY);
    int i = lane < K1 ? Li[q] : (t < nb[q] ? buf->i[q][t] : -1);
    wave_sort64(d, i);
    Ld[q] = lane < K1 ? d : INFINITY;
    Li[q] = lane < K1 ? i : -1;
    th_d[q] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, d), K1 - 1));
    nb[q] = 0;
    __builtin_amdgcn_wave_barrier();
  };
  // the tree rows through a buffer resource: row c of node n at byte
  // offset c * ld * 4 (scalar) + n * 4 (per lane), no 64-bit address math;
  // the host keeps 14 * ld * 4 below 2^31
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)tree, (short)0, (int)(FN_STATE * ld * 4), 0x00020000);
  const int row_bytes = (int)ld * 4;
  float y2max = 0.f;
  const int n0 = ch * chunk;
  const int n1 = min(n0 + chunk, n_nodes);
  // 64 nodes from nb0 on: coordinates and |y|^2 of this lane's node
  auto block = [&](int nb0, const float* y, float yy) {
    const int node = nb0 + lane;
    const bool valid = node < n1;
    y2max = valid ? fmaxf(y2max, yy) : y2max;
#pragma unroll
    for (int q = 0; q < QG; ++q) {
      float d = yy + xx[q];
#pragma unroll
      for (int c = 0; c < FN_STATE; ++c) d = fmaf(xm2[q][c], y[c], d);
      d = valid ? d : INFINITY;
      uint64_t mask = __ballot(d < th_d[q]);
      while (mask) {
        // append the lowest `take` candidates to the buffer
        const int cnt = (int)__popcll(mask), room = CAP - nb[q];
        const int take = cnt < room ? cnt : room;
        const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
        const bool in = ((mask >> lane) & 1ull) && rank < take;
        if (in) {
          buf->d[q][nb[q] + rank] = d;
          buf->i[q][nb[q] + rank] = node;
        }
        mask &= ~__ballot(in);
        nb[q] += take;
        if (nb[q] == CAP) {
          merge(q);
          mask &= __ballot(d < th_d[q]);
        }
      }
    }
  };
  if constexpr (!TILED) {
    for (int nb0 = n0; nb0 < n1; nb0 += WAVE) {
      const int node = nb0 + lane;
      const int nc = node < n1 ? node : n1 - 1;
      float y[FN_STATE];
      float yy = 0.f;
#pragma unroll
      for (int c = 0; c < FN_STATE; ++c) {
        y[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, nc * 4, c * row_bytes, 0));
        yy = fmaf(y[c], y[c], yy);
      }
      block(nb0, y, yy);
    }
  } else {
    const int tid = threadIdx.x;  // 0 .. 255
    for (int t0 = n0; t0 < n1; t0 += KNN_TILE) {
      {
        const int node = t0 + tid;
        const int nc = node < n1 ? node : n1 - 1;
        float yy = 0.f;
#pragma unroll
        for (int c = 0; c < FN_STATE; ++c) {
          const float v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, nc * 4, c * row_bytes, 0));
          tile[tid * KNN_TILE_LD + c] = v;
          yy = fmaf(v, v, yy);
        }
        tile[tid * KNN_TILE_LD + FN_STATE] = yy;
      }
      __syncthreads();
      if (active) {
        const int nt = min(KNN_TILE, n1 - t0);
        for (int sb = 0; sb < nt; sb += WAVE) {
          const float* row = tile + (sb + lane) * KNN_TILE_LD;
          float y[FN_STATE];
#pragma unroll
          for (int c = 0; c < FN_STATE; ++c) y[c] = row[c];
          block(t0 + sb, y, row[FN_STATE]);
        }
      }
      __syncthreads();
    }
    if (!active) return;
  }
#pragma unroll
  for (int q = 0; q < QG; ++q)
    if (nb[q] > 0) merge(q);
  y2max = wave_max(y2max);
#pragma unroll
  for (int q = 0; q < QG; ++q) {
    const int b = grp * QG + q;
    if (b < B) {
      if (lane < K1) {
        const size_t base = ((size_t)b * n_split + ch) * K1;
        out_d[base + lane] = Ld[q];
        out_i[base + lane] = Li[q];
      }
      if (lane == 0) out_y2[(size_t)b * n_split + ch] = y2max;
    }
  }
}

// Matrix-core form: one wavefront per (16 queries, node chunk).  With
// augmented vectors a = (-2 x, |x|^2, 1) and b = (y, 1, |y|^2) (16
// components) the screening key |x|^2 + |y|^2 - 2 x.y is the dot product
// a.b, so a 16 x 16 block of keys (16 queries x 16 nodes) is four
// v_mfma_f32_16x16x4_f32 steps over K = 16.  Operand layout: lane l = 16 r +
// c holds A[c][4 s + r] and B[4 s + r][c] in step s and receives D[4 r + i][c],
// i = 0..3: the keys of queries 4 r + i against node c.  |y|^2 is summed from
// the four lanes that hold a node's coordinates (lane exchanges).  Any order
// of the 16 products and sums stays within the key error bound the merge
// assumes (16 roundings of terms bounded by (|x| + |y|)^2).
// Selection as in the VALU form, per query: a node below the query's
// threshold is appended to its LDS buffer (lanes of a row rank their
// candidates within the row); a query whose buffer would overflow is merged
// first (the 64 entries sorted over the wavefront, K1 kept, threshold
// renewed).  Nodes arrive in increasing index, so the strict test keeps the
// exact FP32 top K1 by (d^2, index), and the chunk lists match the VALU form's
// key for key whenever the FP32 keys agree; the band the merge re-ranks in
// FP64 covers any difference.
constexpr int KNN_QB = 16;
typedef float knn_v4f __attribute__((ext_vector_type(4)));

// Sorts the first n entries of an LDS buffer of 64 (d^2, index) pairs over
// the wavefront, writes the K1 smallest back in order and returns the K1-th
// key (+inf when fewer than K1 entries).
template <int K1>
__device__ __noinline__ float knn_sort_buffer(float* bd, int32_t* bi, int n) {
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_wave_barrier();
  float d = lane < n ? bd[lane] : INFINITY;
  int idx = lane < n ? bi[lane] : -1;
  wave_sort64(d, idx);
  if (lane < K1) {
    bd[lane] = d;
    bi[lane] = idx;
  }
  __builtin_amdgcn_wave_barrier();
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, d), K1 - 1));
}


template <int K1>
__device__ __forceinline__ void knn_scan_mfma_item(const float* __restrict__ tree, int64_t ld, int n_nodes,
                                   const float* __restrict__ qs, int B, int grp, int ch,
                                   int n_split, int chunk, float* __restrict__ out_d,
                                   int32_t* __restrict__ out_i, float* __restrict__ out_y2,
                                   KnnBuf<KNN_QB>* buf) {
  static_assert(K1 + 16 <= WAVE, "a merge must leave room for one 16-node block");
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, row = lane >> 4;
  // A operand: query grp * 16 + col (padding queries repeat the last one)
  float a[4];
  {
    const float* x = qs + (size_t)min(grp * KNN_QB + col, B - 1) * FN_STATE;
    float xx = 0.f;
#pragma unroll
    for (int c = 0; c < FN_STATE; ++c) xx = fmaf(x[c], x[c], xx);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + row;
      a[s] = k < FN_STATE ? -2.f * x[k] : (k == FN_STATE ? xx : 1.f);
    }
  }
  // per lane, for its queries 4 row + i: threshold, buffer count, and
  // whether the buffer holds entries not yet merged
  float thv[4];
  int nbv[4];
  bool dirty[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    thv[i] = INFINITY;
    nbv[i] = 0;
    dirty[i] = true;  // never merged: the final merge sorts (or pads) the list
  }
  // query 4 g + i: buffer sorted over the wavefront (one out-of-line copy
  // of the sort for all call sites), K1 kept, threshold and counts renewed
  // in row g
  auto merge = [&](int g, int i) {
    const int q = 4 * g + i;
    const int nbq = __builtin_amdgcn_readlane(nbv[i], 16 * g);
    const float th = knn_sort_buffer<K1>(buf->d[q], buf->i[q], nbq);
    if (row == g) {
      thv[i] = th;
      nbv[i] = K1;
      dirty[i] = false;
    }
  };
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)tree, (short)0, (int)(FN_STATE * ld * 4), 0x00020000);
  const int row_bytes = (int)ld * 4;
  // step s reads coordinate 4 s + row; step 3 of rows 2 and 3 (the |x|^2 and
  // 1 components) reads row 13 and replaces it
  const int voff_r = row * row_bytes, voff_r3 = min(row, 1) * row_bytes;
  const int n0 = ch * chunk;
  const int n1 = min(n0 + chunk, n_nodes);
  float y2max = 0.f;
  // node nb0 + 16 j + col at byte offset 4 (nb0 + col) + 64 j of its row;
  // in the chunk's last block (wave-uniform test) the nodes past the chunk
  // read its last node and get |y|^2 = +inf below
  for (int nb0 = n0; nb0 < n1; nb0 += WAVE) {
    float bv[4][4];
    const bool tail = nb0 + WAVE > n1;
    if (!tail) {
      const int vn = (nb0 + col) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int s = 0; s < 3; ++s)
          bv[j][s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                   rs, vn + voff_r + 64 * j, 4 * s * row_bytes, 0));
        bv[j][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                 rs, vn + voff_r3 + 64 * j, 12 * row_bytes, 0));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int vn = min(nb0 + 16 * j + col, n1 - 1) * 4;
#pragma unroll
        for (int s = 0; s < 3; ++s)
          bv[j][s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                   rs, vn + voff_r, 4 * s * row_bytes, 0));
        bv[j][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                 rs, vn + voff_r3, 12 * row_bytes, 0));
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float p = bv[j][0] * bv[j][0];
      p = fmaf(bv[j][1], bv[j][1], p);
      p = fmaf(bv[j][2], bv[j][2], p);
      p = row < 2 ? fmaf(bv[j][3], bv[j][3], p) : p;
      // sum over the four rows; a lane and its partner add the same two
      // values, so the four lanes of a node hold the same |y|^2
      const float t = p + __builtin_bit_cast(float, lane_xor<16>(__builtin_bit_cast(int, p)));
      const float yy = t + __builtin_bit_cast(float, lane_xor<32>(__builtin_bit_cast(int, t)));
      const bool valid = !tail || nb0 + 16 * j + col < n1;
      y2max = valid ? fmaxf(y2max, yy) : y2max;
      // a node past the chunk gets |y|^2 = +inf: every key of it is +inf
      const float y15 = valid ? yy : INFINITY;
      bv[j][3] = row < 2 ? bv[j][3] : (row == 2 ? 1.f : y15);
    }
    knn_v4f acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = knn_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv[j][s], acc[j], 0, 0, 0);
    bool any = false;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) any |= acc[j][i] < thv[i];
    if (__ballot(any) == 0) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float d = acc[j][i];
        uint64_t m = __ballot(d < thv[i]);
        if (m == 0) continue;
        uint32_t gm = (uint32_t)(m >> (16 * row)) & 0xffffu;
        // rows whose query would overflow its buffer: merge those first
        uint64_t over = __ballot(nbv[i] + (int)__popc(gm) > WAVE) & 0x0001000100010001ull;
        if (over) {
          while (over) {
            const int g = (int)__builtin_ctzll(over) >> 4;
            over &= over - 1;
            merge(g, i);
          }
          m = __ballot(d < thv[i]);
          gm = (uint32_t)(m >> (16 * row)) & 0xffffu;
        }
        if (d < thv[i]) {
          const int slot = nbv[i] + (int)__popc(gm & ((1u << col) - 1u));
          buf->d[4 * row + i][slot] = d;
          buf->i[4 * row + i][slot] = nb0 + 16 * j + col;
        }
        nbv[i] += (int)__popc(gm);
        dirty[i] = dirty[i] || gm != 0;
      }
    }
  }
  // final merges: every query with unmerged entries (or never merged)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint64_t pend = __ballot(dirty[i]) & 0x0001000100010001ull;
    while (pend) {
      const int g = (int)__builtin_ctzll(pend) >> 4;
      pend &= pend - 1;
      merge(g, i);
    }
  }
  y2max = wave_max(y2max);
  __builtin_amdgcn_wave_barrier();
  for (int e = lane; e < KNN_QB * K1; e += WAVE) {
    const int q = e / K1, t = e - q * K1;
    const int b = grp * KNN_QB + q;
    if (b < B) {
      const size_t base = ((size_t)b * n_split + ch) * K1;
      out_d[base + t] = buf->d[q][t];
      out_i[base + t] = buf->i[q][t];
    }
  }
  if (lane < KNN_QB && grp * KNN_QB + lane < B)
    out_y2[(size_t)(grp * KNN_QB + lane) * n_split + ch] = y2max;
}

// FP64 squared distance, summed in the reference order with separately
// rounded operations.
__device__ __forceinline__ double exact_d2(const float* __restrict__ tree, int64_t ld, int node,
                                           const double* x) {
  double d = 0.0;
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) {
    const double t = __dsub_rn(x[c], (double)tree[(size_t)c * ld + node]);
    d = __dadd_rn(d, __dmul_rn(t, t));
  }
  return d;
}

__device__ __forceinline__ unsigned long long dkey(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// wave-wide argmin over (d64, idx) keys held one per lane; returns the
// winning lane's (d, idx) in every lane.
__device__ __forceinline__ void wave_argmin(double d, int idx, double& wd, int& wi) {
  unsigned long long k = dkey(d);
  unsigned long long m = k;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long v = __shfl_xor(m, o);
    m = v < m ? v : m;
  }
  unsigned mi = (k == m) ? (unsigned)idx : 0xffffffffu;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned v = __shfl_xor(mi, o);
    mi = v < mi ? v : mi;
  }
  wd = __longlong_as_double((long long)m);
  wi = (int)mi;
}

// Sorts the 64 lanes' (key, index) pairs ascending, key first, then the
// index as unsigned (bitonic network; equal pairs stay put).
template <int K, int J>
__device__ __forceinline__ void bitonic_stage2(uint64_t& key, int& idx) {
  const int lane = threadIdx.x & 63;
  const uint64_t ok = ((uint64_t)(uint32_t)lane_xor<J>((int)(key >> 32)) << 32) |
                      (uint32_t)lane_xor<J>((int)(uint32_t)key);
  const int oi = lane_xor<J>(idx);
  const bool o_less = ok < key || (ok == key && (unsigned)oi < (unsigned)idx);
  const bool o_more = key < ok || (ok == key && (unsigned)idx < (unsigned)oi);
  const bool want_min = ((lane & J) == 0) == ((lane & K) == 0);
  if (want_min ? o_less : o_more) {
    key = ok;
    idx = oi;
  }
}
template <int K, int J>
__device__ __forceinline__ void bitonic_merge2(uint64_t& key, int& idx) {
  bitonic_stage2<K, J>(key, idx);
  if constexpr (J > 1) bitonic_merge2<K, J / 2>(key, idx);
}
__device__ __forceinline__ void wave_sort64_2(uint64_t& key, int& idx) {
  bitonic_merge2<2, 1>(key, idx);
  bitonic_merge2<4, 2>(key, idx);
  bitonic_merge2<8, 4>(key, idx);
  bitonic_merge2<16, 8>(key, idx);
  bitonic_merge2<32, 16>(key, idx);
  bitonic_merge2<64, 32>(key, idx);
}

// Exact FP64 rescan of the whole tree for query b (x: its state in FP64):
// each lane keeps a sorted list of its k best, then k rounds of wave argmin
// over the list heads.
__device__ void knn_rescan_query(const float* __restrict__ tree, int64_t ld, int n_nodes,
                                 const double* x, int b, int k, int32_t* __restrict__ out_idx,
                                 float* __restrict__ out_d2) {
  const int lane = threadIdx.x & 63;
  double ld_d[FN_MAX_K];
  int ld_i[FN_MAX_K];
  for (int r = 0; r < k; ++r) {
    ld_d[r] = INFINITY;
    ld_i[r] = 0x7fffffff;
  }
  for (int n = lane; n < n_nodes; n += 64) {
    const double d = exact_d2(tree, ld, n, x);
    if (d < ld_d[k - 1]) {  // a lane's nodes come in increasing index
      int r = k - 1;
      while (r > 0 && d < ld_d[r - 1]) {
        ld_d[r] = ld_d[r - 1];
        ld_i[r] = ld_i[r - 1];
        --r;
      }
      ld_d[r] = d;
      ld_i[r] = n;
    }
  }
  int head = 0;
  for (int r = 0; r < k; ++r) {
    const double hd = head < k ? ld_d[head] : INFINITY;
    const int hi = head < k ? ld_i[head] : 0x7fffffff;
    double wd;
    int wi;
    wave_argmin(hd, hi, wd, wi);
    if (wi != 0x7fffffff && wi == hi) ++head;
    if (wi == 0x7fffffff) {
      wd = INFINITY;
      wi = -1;
    }
    if (lane == 0) {
      out_idx[(size_t)b * k + r] = wi;
      if (out_d2) out_d2[(size_t)b * k + r] = (float)wd;
    }
  }
}

// Smallest 64 of two ascending 64-lane lists (a in every lane, b in every
// lane): a's first 32 keys in lanes 0..31 and b's first 32 in reverse in
// lanes 32..63 form a bitonic sequence, and one merge sorts it.  Enough for
// the k <= 32 smallest.
__device__ __forceinline__ void wave_merge_heads(uint64_t& a, int& ai, uint64_t b, int bi) {
  const int lane = threadIdx.x & 63;
  const int src = (63 - lane) << 2;
  const uint64_t rb = ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(b >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)b);
  const int rbi = __builtin_amdgcn_ds_bpermute(src, bi);
  if (lane >= 32) {
    a = rb;
    ai = rbi;
  }
  bitonic_merge2<64, 32>(a, ai);
}

// Merge of one query whose chunk lists hold at most 128 entries in all
// (n_split * K1 <= 128): one or two entries per lane; the FP32 k-th key
// comes from sorts of the 64-bit keys, the FP64 ranking of the band from
// sorts of (d64, index) -- the same result as the k rounds of argmin of the
// general merge.  No LDS.
template <int K1>
__device__ void knn_merge_small(const float* __restrict__ tree, int64_t ld, int n_nodes,
                                const float* __restrict__ qs, int b, int k, int n_split,
                                const float* __restrict__ in_d, const int32_t* __restrict__ in_i,
                                const float* __restrict__ in_y2, int32_t* __restrict__ out_idx,
                                float* __restrict__ out_d2) {
  const int lane = threadIdx.x & 63;
  double x[FN_STATE];
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) x[c] = (double)qs[(size_t)b * FN_STATE + c];
  const int total = n_split * K1;
  const bool two = total > WAVE;
  const float* D = in_d + (size_t)b * total;
  const int32_t* I = in_i + (size_t)b * total;
  // entry e0 = lane and (two lists) e1 = lane + 64
  const int e1 = lane + WAVE;
  int i0 = lane < total ? I[lane] : -1, i1 = two && e1 < total ? I[e1] : -1;
  float d0 = i0 >= 0 ? D[lane] : INFINITY, d1 = i1 >= 0 ? D[e1] : INFINITY;
  // (a) FP32 k-th smallest key over all entries
  uint64_t ka = knn_key(d0, i0);
  int ia = 0;
  wave_sort64_2(ka, ia);
  if (two) {
    uint64_t kb = knn_key(d1, i1);
    int ib = 0;
    wave_sort64_2(kb, ib);
    wave_merge_heads(ka, ia, kb, ib);
  }
  const uint64_t th = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(ka >> 32), k - 1) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ka, k - 1);
  const float th_d = knn_key_d(th);
  const int th_i = (int)(uint32_t)th;
  // error bound of the screening distances (as in the general merge)
  float y2 = 0.f;
  for (int c2 = lane; c2 < n_split; c2 += 64) y2 = fmaxf(y2, in_y2[(size_t)b * n_split + c2]);
  y2 = wave_max(y2);
  double xn = 0.0;
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) xn += x[c] * x[c];
  const float rad = (float)sqrt(xn) + sqrtf(y2);
  const float eps = KNN_EPS * rad * rad;
  const float band = th_i < 0 ? INFINITY : th_d + 2.f * eps + fabsf(th_d) * KNN_BAND + 1e-30f;
  // (b) a chunk whose last entry is in the band may hold more in-band nodes
  const bool over0 = lane < total && lane % K1 == K1 - 1 && i0 >= 0 && d0 <= band;
  const bool over1 = e1 < total && e1 % K1 == K1 - 1 && i1 >= 0 && d1 <= band;
  if (__any(over0 || over1)) {
    knn_rescan_query(tree, ld, n_nodes, x, b, k, out_idx, out_d2);
    return;
  }
  // (c) FP64 re-rank of the band: sorts of (d64, index); entries outside
  // the band rank last (+inf, max index).  d >= 0, so the bit order of the
  // doubles is their value order.
  const bool in0 = i0 >= 0 && d0 <= band, in1 = i1 >= 0 && d1 <= band;
  uint64_t ga = (uint64_t)__double_as_longlong(in0 ? exact_d2(tree, ld, i0, x) : INFINITY);
  int gia = in0 ? i0 : 0x7fffffff;
  wave_sort64_2(ga, gia);
  if (two) {
    uint64_t gb = (uint64_t)__double_as_longlong(in1 ? exact_d2(tree, ld, i1, x) : INFINITY);
    int gib = in1 ? i1 : 0x7fffffff;
    wave_sort64_2(gb, gib);
    wave_merge_heads(ga, gia, gb, gib);
  }
  if (lane < k) {
    const bool ok = gia != 0x7fffffff;
    out_idx[(size_t)b * k + lane] = ok ? gia : -1;
    if (out_d2) out_d2[(size_t)b * k + lane] = ok ? (float)__longlong_as_double((long long)ga) : INFINITY;
  }
}

template <int K1>
__device__ void knn_merge_query(const float* __restrict__ tree, int64_t ld, int n_nodes,
                                const float* __restrict__ qs, int b, int k, int n_split,
                                const float* __restrict__ in_d, const int32_t* __restrict__ in_i,
                                const float* __restrict__ in_y2, int32_t* __restrict__ out_idx,
                                float* __restrict__ out_d2) {
  const int lane = threadIdx.x & 63;
  double x[FN_STATE];
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) x[c] = (double)qs[(size_t)b * FN_STATE + c];
  const int total = n_split * K1;
  const float* D = in_d + (size_t)b * total;
  const int32_t* I = in_i + (size_t)b * total;

  // (a) FP32 k-th smallest key over all chunk lists (each chunk's K1 >= k
  // smallest keys, so this is the k-th smallest screening key overall)
  float th_d = -1.f;
  int th_i = -1;
  for (int r = 0; r < k; ++r) {
    float bd = INFINITY;
    int bi = -1;
    for (int e = lane; e < total; e += 64) {
      const float d = D[e];
      const int i = I[e];
      if (i < 0) continue;
      const bool after = th_i < 0 ? true : key_less(th_d, th_i, d, i);
      if (after && key_less(d, i, bd, bi)) {
        bd = d;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float od = __shfl_xor(bd, o);
      const int oi = __shfl_xor(bi, o);
      if (key_less(od, oi, bd, bi)) {
        bd = od;
        bi = oi;
      }
    }
    if (bi < 0) break;  // fewer than k nodes in total
    th_d = bd;
    th_i = bi;
  }
  // absolute error bound of the FP32 screening distances of this query:
  // 4e-6 (|x| + max |y|)^2, max over every chunk (the whole tree)
  float y2 = 0.f;
  for (int c2 = lane; c2 < n_split; c2 += 64) y2 = fmaxf(y2, in_y2[(size_t)b * n_split + c2]);
  y2 = wave_max(y2);
  double xn = 0.0;
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) xn += x[c] * x[c];
  const float rad = (float)sqrt(xn) + sqrtf(y2);
  const float eps = KNN_EPS * rad * rad;
  // every exact top-k node has a screening key within th + 2 eps
  const float band = th_i < 0 ? INFINITY : th_d + 2.f * eps + fabsf(th_d) * KNN_BAND + 1e-30f;

  // (b) a chunk whose last entry is inside the band may hold more in-band
  // nodes than its list
  int over = 0;
  for (int e = lane; e < total; e += 64)
    if (e % K1 == K1 - 1 && I[e] >= 0 && D[e] <= band) over = 1;
  over = __any(over);

  if (!over) {
    // (c) FP64 re-rank of the band (computed once into LDS), then k rounds
    // of wave argmin over (d64, index)
    __shared__ double s_d[KNN_MAX_SPLIT * (FN_MAX_K + 1)];
    for (int e = lane; e < total; e += 64) {
      const int i = I[e];
      const bool in = i >= 0 && D[e] <= band;
      s_d[e] = in ? exact_d2(tree, ld, i, x) : INFINITY;
    }
    __syncthreads();
    double prev_d = -1.0;
    int prev_i = -1;
    for (int r = 0; r < k; ++r) {
      double bd = INFINITY;
      int bi = 0x7fffffff;
      for (int e = lane; e < total; e += 64) {
        const double d = s_d[e];
        if (!(d < INFINITY)) continue;
        const int i = I[e];
        const bool after = prev_i < 0 || d > prev_d || (d == prev_d && i > prev_i);
        if (after && (d < bd || (d == bd && i < bi))) {
          bd = d;
          bi = i;
        }
      }
      double wd;
      int wi;
      wave_argmin(bd, bi, wd, wi);
      if (wi == 0x7fffffff) {
        wd = INFINITY;
        wi = -1;
      } else {
        prev_d = wd;
        prev_i = wi;
      }
      if (lane == 0) {
        out_idx[(size_t)b * k + r] = wi;
        if (out_d2) out_d2[(size_t)b * k + r] = (float)wd;
      }
    }
  } else {
    knn_rescan_query(tree, ld, n_nodes, x, b, k, out_idx, out_d2);
  }
}

constexpr int KNN_QG = 4;  // queries per scan wavefront

}  // namespace fn
