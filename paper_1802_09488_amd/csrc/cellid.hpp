// cellid.hpp -- cube-face / quadtree / Hilbert cell ids (Section II, S2
// paragraph; Fig. 2): 3 face bits, one bit pair per level (30 levels), a
// marker bit, zeros. The paper leaves the face numbering, (u, v) axes,
// uv -> st transform and curve orientation open and only needs a child's id
// to extend its parent's prefix. This library's choice:
//   x = cos(lat) cos(lng), y = cos(lat) sin(lng), z = sin(lat);
//   axis a = argmax |c| (ties to the lower axis), face = a or a + 3 (negative);
//   u = c[(a+1)%3] / |c[a]|, v = c[(a+2)%3] / |c[a]|;
//   s = st(u), t = st(v), st(w) = (1 + w) / 2 (linear; S2 offers it too);
//   i = clamp(floor(2^30 s)), j = clamp(floor(2^30 t));
//   Hilbert digit per level from the quadrant (rx, ry) as (3 rx) xor ry,
//   sub-squares with ry = 0 reflected (rx = 1) and transposed.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#ifndef ACT_HD
#define ACT_HD __host__ __device__ __forceinline__
#endif

namespace act {

constexpr int kMaxLevel = 30;
constexpr double kTwo30 = 1073741824.0;

ACT_HD double st_from_uv(double u) { return 0.5 * (1.0 + u); }

ACT_HD double uv_from_st(double s) { return 2.0 * s - 1.0; }

// Hilbert state machine. State = (swap s, flip f): the transform taking the
// original sub-square coordinates to the curve's canonical frame (flip =
// complement both coordinates, swap = exchange them; they commute). Per
// level: (a, b) = state applied to the quadrant bits, digit = (3a) ^ b, and
// when b == 0 the state absorbs "reflect if a, then transpose".
// The 4-level table maps (state << 8 | i_nibble << 4 | j_nibble) to
// (digits (8 bits) | next_state << 8).
inline void hilbert_table4(uint16_t table[1024]) {
  for (int state = 0; state < 4; state++)
    for (int byte = 0; byte < 256; byte++) {
      int s = state & 1, f = state >> 1;
      int xi = byte >> 4, yj = byte & 15, digits = 0;
      for (int k = 3; k >= 0; k--) {
        int x = (xi >> k) & 1, y = (yj >> k) & 1;
        int a = x ^ f, b = y ^ f;
        if (s) {
          int tmp = a;
          a = b;
          b = tmp;
        }
        digits = (digits << 2) | ((3 * a) ^ b);
        if (b == 0) {
          s ^= 1;
          f ^= a;
        }
      }
      table[state * 256 + byte] = (uint16_t)(digits | ((s | (f << 1)) << 8));
    }
}

// Hilbert position (60 bits) of a leaf (i, j), i, j < 2^30, using the
// 4-level table. The coordinates are processed as 32-bit values: the two
// leading zero levels leave the state unchanged and contribute zero digits.
template <typename Table>
ACT_HD uint64_t hilbert_pos30(uint32_t i, uint32_t j, const Table &tab) {
  uint32_t state = 0;
  uint64_t d = 0;
#pragma unroll
  for (int sh = 28; sh >= 0; sh -= 4) {
    uint32_t idx = (state << 8) | (((i >> sh) & 15u) << 4) | ((j >> sh) & 15u);
    uint32_t e = tab[idx];
    d = (d << 8) | (e & 255u);
    state = e >> 8;
  }
  return d;
}

// Cell id of the level-`level` cell (i, j) (coordinates of that level).
template <typename Table>
inline uint64_t cell_id(int face, int level, uint32_t i, uint32_t j, const Table &tab) {
  int sh = kMaxLevel - level;
  uint64_t pos = hilbert_pos30(i << sh, j << sh, tab) >> (2 * sh);
  return ((uint64_t)face << 61) | (pos << (2 * sh + 1)) | (1ull << (2 * sh));
}

// Face-relative 60-bit key of a cell: its Hilbert position left-aligned to
// 30 levels (the leaf position of its first descendant).
inline uint64_t cell_key(uint64_t id) {
  uint64_t lsb = id & (~id + 1);
  return ((id & ((1ull << 61) - 1)) - lsb) >> 1;
}

inline int cell_level(uint64_t id) { return kMaxLevel - __builtin_ctzll(id) / 2; }

}  // namespace act
