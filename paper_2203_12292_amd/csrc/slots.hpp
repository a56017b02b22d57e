// Geometry of the 27 entity slots of a hexahedron and the hanging-node line
// rule, shared by host set-up and device kernels.
//
// Slots: 0-7 vertices (a + 2b + 4c), 8-11 edges along x (8 + b + 2c),
// 12-15 edges along y (12 + a + 2c), 16-19 edges along z (16 + a + 2b),
// 20-21 faces normal to x (20 + a), 22-23 normal to y (22 + b), 24-25 normal
// to z (24 + c), 26 interior; a, b, c in {0, 1} select the low/high side.
//
// Within an entity, DoFs are ordered over the entity's interior node indices
// with x fastest, then y, then z.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfmg {

// side of slot s along axis d: 0 / 1 (at node 0 / node k), -1 (extends)
__host__ __device__ constexpr int slot_side(int s, int d) {
  return s < 8 ? ((s >> d) & 1)
         : s < 12 ? (d == 0 ? -1 : d == 1 ? ((s - 8) & 1) : (((s - 8) >> 1) & 1))
         : s < 16 ? (d == 1 ? -1 : d == 0 ? ((s - 12) & 1) : (((s - 12) >> 1) & 1))
         : s < 20 ? (d == 2 ? -1 : d == 0 ? ((s - 16) & 1) : (((s - 16) >> 1) & 1))
         : s < 22 ? (d == 0 ? (s - 20) : -1)
         : s < 24 ? (d == 1 ? (s - 22) : -1)
         : s < 26 ? (d == 2 ? (s - 24) : -1)
                  : -1;
}

// slot of node (a, b, c), 0 <= a, b, c <= k
__host__ __device__ constexpr int node_slot(int a, int b, int c, int k) {
  int sa = a == 0 ? 0 : a == k ? 1 : -1;
  int sb = b == 0 ? 0 : b == k ? 1 : -1;
  int sc = c == 0 ? 0 : c == k ? 1 : -1;
  int ext = (sa < 0) + (sb < 0) + (sc < 0);
  if (ext == 0) return sa + 2 * sb + 4 * sc;
  if (ext == 1) return sa < 0 ? 8 + sb + 2 * sc : sb < 0 ? 12 + sa + 2 * sc : 16 + sa + 2 * sb;
  if (ext == 2) return sa >= 0 ? 20 + sa : sb >= 0 ? 22 + sb : 24 + sc;
  return 26;
}

// offset of node (a, b, c) inside its slot's entity
__host__ __device__ constexpr int node_offset(int a, int b, int c, int k) {
  int km = k - 1;
  int ea = (a != 0 && a != k), eb = (b != 0 && b != k), ec = (c != 0 && c != k);
  int off = 0, stride = 1;
  if (ea) { off += (a - 1) * stride; stride *= km; }
  if (eb) { off += (b - 1) * stride; stride *= km; }
  if (ec) { off += (c - 1) * stride; }
  return off;
}

__host__ __device__ constexpr int slot_size(int s, int k) {
  int km = k - 1;
  return s < 8 ? 1 : s < 20 ? km : s < 26 ? km * km : km * km * km;
}

// Operator kernels: a cell is handled by n^2 lanes of one wavefront (one
// lane per line of n nodes), cells_per_wave(n) = floor(64 / n^2) cells per
// wavefront, BATCH_WAVES wavefronts per block.
#ifndef MFMG_BATCH_WAVES
#define MFMG_BATCH_WAVES 8
#endif
constexpr int BATCH_WAVES = MFMG_BATCH_WAVES;
__host__ __device__ constexpr int cells_per_wave(int n) { return 64 / (n * n); }

// Cell batches of the operator: a batch's DoFs are staged in LDS (input and
// accumulated output) next to the per-wave work buffers, within
// BATCH_LDS_BYTES per block (sized for FP64).  batch_mcap(k) bounds the DoFs a
// batch touches.  Behind them sits a block of batch_zero_entries(k) entries:
// zeros in the input and a discarded area in the output, where absent
// (Dirichlet) entities and lanes without a cell point, so that gather and
// scatter need no branches.
#ifndef MFMG_BATCH_LDS_BYTES
#define MFMG_BATCH_LDS_BYTES 81920
#endif
constexpr int BATCH_LDS_BYTES = MFMG_BATCH_LDS_BYTES;
constexpr int BATCH_MAX_CELLS = 1024;
// From degree 5 on, the batch's cell metadata (64 B per cell) is staged in
// LDS too, for at most two cell groups of the block per batch.
__host__ __device__ constexpr bool batch_meta_in_lds(int k) { return k >= 5; }
__host__ __device__ constexpr int batch_max_cells(int k) {
  return batch_meta_in_lds(k) ? 2 * BATCH_WAVES * cells_per_wave(k + 1) : BATCH_MAX_CELLS;
}
#ifndef MFMG_BATCH_QUANTIZE
#define MFMG_BATCH_QUANTIZE 1
#endif
constexpr bool BATCH_QUANTIZE = MFMG_BATCH_QUANTIZE != 0;
// persistent operator blocks per resident block slot of the device
#ifndef MFMG_BATCH_GRID_FACTOR
#define MFMG_BATCH_GRID_FACTOR 2
#endif
constexpr int BATCH_GRID_FACTOR = MFMG_BATCH_GRID_FACTOR;
__host__ __device__ constexpr int batch_zero_entries(int k) { return k > 1 ? (k - 1) * (k - 1) * (k - 1) : 1; }
__host__ __device__ constexpr int batch_work_bytes(int k) {
  // one n^3 buffer per cell of every wavefront plus a spare one for lanes
  // without a cell, the hanging-interpolation matrices of both halves and the
  // staged cell metadata
  return (BATCH_WAVES * cells_per_wave(k + 1) + 1) * (k + 1) * (k + 1) * (k + 1) * 8 + 2 * (k + 1) * (k + 1) * 8 +
         (batch_meta_in_lds(k) ? batch_max_cells(k) * 64 : 0);
}
__host__ __device__ constexpr int batch_mcap(int k) {
  return ((BATCH_LDS_BYTES - batch_work_bytes(k)) / 16 - batch_zero_entries(k)) / 64 * 64;
}

// Mask bits.
__host__ __device__ inline int mask_sub(uint32_t m, int d) { return (m >> d) & 1; }
__host__ __device__ inline int mask_face(uint32_t m, int d) { return (m >> (3 + d)) & 1; }
__host__ __device__ inline int mask_edge(uint32_t m, int d) { return (m >> (6 + d)) & 1; }
__host__ __device__ inline int mask_level(uint32_t m) { return (m >> 16) & 0xff; }
__host__ __device__ inline bool mask_hanging(uint32_t m) { return (m & 0x1f8u) != 0; }
// Diffusion coefficient of the cell (constant per cell, positive) as a
// bfloat16 in the mask bits the layout leaves free: exponent in bits 24-31,
// the 7 stored mantissa bits in bits 9-15.
__host__ __device__ inline float mask_coef(uint32_t m) {
  const uint32_t bits = ((m >> 24) << 23) | (((m >> 9) & 0x7fu) << 16);
  return __builtin_bit_cast(float, bits);
}
constexpr uint32_t MASK_COEF_BITS = 0xff00fe00u;
// transfer valence byte: owner flag (the low bits count the groups)
constexpr uint8_t TRANSFER_OWNER = 0x80;
// The mask bits of a coefficient c in [1e-30, 1e30]: c rounded to 8
// significant bits (bfloat16), ties to even, from the bits of the double.
__host__ __device__ inline uint32_t coef_bits(double c) {
  const uint64_t b = __builtin_bit_cast(uint64_t, c);
  int e = static_cast<int>((b >> 52) & 0x7ff) - 1023 + 127;  // float exponent field
  const uint64_t frac = b & ((uint64_t(1) << 52) - 1);
  uint32_t m7 = static_cast<uint32_t>(frac >> 45);
  const uint64_t rest = frac & ((uint64_t(1) << 45) - 1), half = uint64_t(1) << 44;
  if (rest > half || (rest == half && (m7 & 1u))) ++m7;
  if (m7 == 0x80u) {  // rounded up to the next power of two
    m7 = 0;
    ++e;
  }
  return static_cast<uint32_t>(e) << 24 | m7 << 9;
}

// Is the line along axis d through local node indices (p, q) of the other two
// axes (in increasing axis order) interpolated by the hanging-node rule?
// Lines of a hanging face normal to e (e != d) at the face's node index, and
// the hanging edge along d itself.
__host__ __device__ inline bool hanging_line(uint32_t m, int d, int p, int q, int k) {
  const int e = d == 0 ? 1 : 0;
  const int f = d == 2 ? 1 : 2;
  const bool pe = p == mask_sub(m, e) * k;
  const bool qf = q == mask_sub(m, f) * k;
  return (mask_face(m, e) && pe) || (mask_face(m, f) && qf) || (mask_edge(m, d) && pe && qf);
}

// Is slot s constrained (its entity replaced by the parent's entity)?
__host__ __device__ inline bool slot_hanging(uint32_t m, int s) {
  for (int d = 0; d < 3; ++d)
    if (mask_face(m, d) && slot_side(s, d) == mask_sub(m, d)) return true;
  for (int d = 0; d < 3; ++d) {
    const int e = d == 0 ? 1 : 0;
    const int f = d == 2 ? 1 : 2;
    if (mask_edge(m, d) && slot_side(s, e) == mask_sub(m, e) && slot_side(s, f) == mask_sub(m, f))
      return true;
  }
  return false;
}

}  // namespace mfmg
