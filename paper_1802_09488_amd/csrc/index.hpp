// index.hpp -- host-side representation of a built index and the layout of
// its device image (shared by the builder and the GPU runtime).
//
// Adaptive Cell Trie (Section III-C, Fig. 7): nodes of 256 tagged 8-byte
// entries (fanout 256 = 4 cell levels per node). Tag = two low bits:
//   00  child pointer: node index << 2; the value 0 is the sentinel
//       (false hit) -- node 0 is reserved and never referenced;
//   01  one inlined reference: bits 2..32 = polygon id << 1 | interior;
//   10  two inlined references: bits 2..32 and 33..63, ascending ids;
//   11  lookup-table word offset << 2.
// Lookup table: one uint32 array; each list is
//   n_true, true ids..., n_cand, candidate ids... (ids ascending per part);
//   in exact mode a cell with candidates always has its own list, followed
//   by n_cand word offsets (into the same array) of the candidates'
//   cell-local refinement records, which follow right after.
// Per face: a root node, the common prefix shared by every indexed cell on
// the face (prefix level Lp), and the alignment of node levels: the root
// covers levels Lp+1..Lp+4, its children Lp+5..Lp+8, and so on (the
// per-face common prefix of Section IV-B2 / Listing 4 with the level
// granularity g = 4 of Section III-C).
//
// Key: the method needs only that a child's key extends its parent's
// (Section II); it does not depend on the curve. The trie is keyed by the
// cell's quadtree path: a node covering levels L+1..L+4 indexes its 256
// entries by (4 bits of i, 4 bits of j) below level L, i.e. entry
// 16 * ni + nj. The nodes, their contents and depths are those of a trie
// over the Hilbert-ordered cell ids; only the order of entries inside a node
// differs. A probe forms each node's key byte from (i, j) directly, with no
// sequential curve state.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/act.h"

namespace act {

constexpr uint64_t kTagMask = 3;
constexpr uint64_t kTagPtr = 0, kTagOne = 1, kTagTwo = 2, kTagLut = 3;

struct FaceRoot {
  int32_t root = -1;      // node index, -1 if the face has no cells
  int32_t plevel = 0;     // prefix level Lp
  uint32_t pi = 0, pj = 0;  // the common prefix: (i, j) >> (30 - Lp)
  int32_t depth = 0;      // number of node levels below the prefix
};

// Entry of (leaf coordinates i, j) in the node whose levels end `sh` bits
// above the leaf level.
inline __host__ __device__ uint32_t node_slot(uint32_t i, uint32_t j, int sh) {
  return (((i >> sh) & 15u) << 4) | ((j >> sh) & 15u);
}

struct HostIndex {
  int32_t mode = ACT_EXACT;
  double precision_m = 0;
  int32_t max_level = 20;
  int32_t n_polys = 0;

  FaceRoot faces[6];
  std::vector<uint64_t> nodes;   // 256 entries per node, node 0 reserved
  std::vector<uint32_t> lut;

  // polygon store (x = lng, y = lat)
  std::vector<int32_t> poly_edge_off;  // n_polys + 1
  std::vector<double> poly_origin;     // 2 per polygon (x, y)
  std::vector<float> poly_m;           // largest |translated fp32 coordinate|
  std::vector<float> edges32;          // 4 per edge, translated, lower endpoint first
  std::vector<double> edges64;         // 4 per edge: ax ay bx by
  // exact mode: words of cell-local refinement records (stored in `lut`
  // after their cell's list)
  int64_t local_words = 0;
  // ACT_GEOM_SPHERE: edges are great-circle arcs; the normal a x b of each
  // edge's great circle (3 doubles per edge, unit vectors of the endpoints)
  // and the cell margin used (degrees: the build margin plus the largest
  // arc-to-chord distance)
  int32_t geometry = ACT_GEOM_PLANE;
  std::vector<double> normals;
  double margin_deg = 0;

  // statistics
  int64_t n_cells = 0, n_cells_interior_only = 0;
  int32_t max_depth = 0, max_refs = 0, max_cell_level = 0;
  // Nodes are numbered breadth-first: roots occupy indices 1 .. n_d0, the
  // nodes one level below them n_d0+1 .. n_d0+n_d1, so the top two levels
  // are one contiguous run the GPU stages in LDS. Every entry has its high
  // 32 bits zero: the device image keeps 32-bit entries.
  int32_t n_d0 = 0, n_d1 = 0;
  double build_seconds = 0;
  // training (Section III-D): cells split and training points consumed
  int64_t train_splits = 0, train_points_used = 0;
};

// Trie nodes the probe stages in LDS (the top two node levels, as 32-bit
// entries: 1 KiB per node, 64 KiB per block).
constexpr int kLdsTrieNodes = 64;

struct BuildParams {
  int32_t mode;
  double precision_m;
  int32_t max_level;
  int32_t threads;
  int32_t prefix_level;  // -1: automatic
  double margin_deg;
  // training (exact mode): points (lat, lng) and the device-image budget
  const double *train_points = nullptr;
  int64_t n_train = 0;
  int64_t memory_budget = 0;  // bytes, 0 = none
  int32_t train_max_level = 30;
  // stop early (ACT_E_RANGE) once the covering has more cells than this
  // (0 = no limit): a budget check that need not finish the covering
  int64_t cell_limit = 0;
  int32_t geometry = ACT_GEOM_PLANE;
  // per-polygon coverings with cell budgets (exact mode; 0 = the joint
  // subdivision): covering cells (up to max_level) and interior cells (up
  // to max_interior_level)
  int32_t max_covering_cells = 0;
  int32_t max_interior_cells = 256;
  int32_t max_interior_level = 20;
};

// Device bytes of an index image besides its trie nodes and lookup table
// (the polygon store and tables), as the runtime uploads it.
int64_t image_fixed_bytes(int64_t n_polys, int64_t n_edges);

// Device bytes the runtime uploads for this index.
int64_t image_bytes(const HostIndex &h);

// Index files: the host image in a little-endian binary layout (magic,
// version, scalars, then each array as a length and its elements), followed
// by `extra` caller bytes (the launch configuration) and a 64-bit digest of
// everything before it. load_host_index checks the magic, version, lengths
// and digest.
int save_host_index(const HostIndex &h, const void *extra, uint32_t extra_bytes, const char *path,
                    std::string &err);
int load_host_index(const char *path, HostIndex &h, void *extra, uint32_t extra_bytes,
                    std::string &err);

// Builds the host index. Returns ACT_OK or an error code with `err` set.
int build_host_index(const double *verts_latlng, const int64_t *ring_off,
                     const int32_t *poly_ring_off, int32_t n_polys,
                     const BuildParams &bp, HostIndex &out, std::string &err);

// Host trie lookup of a leaf cell (face, i, j): the tagged entry the
// descent ends at.
uint64_t host_lookup(const HostIndex &idx, int face, uint32_t i, uint32_t j);

// Encode one reference list (refs[k] = id << 1 | interior) into a tagged
// entry, deduplicating lists of three or more in `lut` via `dedup`.
struct LutDedup;
LutDedup *lut_dedup_new();
void lut_dedup_free(LutDedup *);
uint64_t encode_refs(const uint32_t *refs, int n, std::vector<uint32_t> &lut, LutDedup *dedup);
// As encode_refs, but always a lookup-table reference.
uint64_t encode_refs_lut(const uint32_t *refs, int n, std::vector<uint32_t> &lut, LutDedup *dedup);

}  // namespace act
