// Device-side layouts shared by the host code and the static kernels.
#pragma once
#include <stdint.h>

namespace wdf {

// One inner node on a group's path.
struct PathNode {
  float thr;        // x < thr goes left
  int32_t feat;     // split feature
  uint8_t dl;       // NaN goes left when nonzero
  uint8_t dir;      // 0: the group's path continues to the left child, 1: right
  uint8_t merge;    // index of the node's feature among the path's distinct features
  uint8_t first;    // 1 when this is the first node of the path carrying the feature
};

// A group: two sibling leaves (pair) or one leaf whose sibling is an inner node
// (single).  A pair's pattern is the left leaf's; the right leaf's is p ^ 1.
struct Group {
  int32_t tree;
  int32_t depth;      // inner nodes on the path, 0..8
  int32_t dprime;     // distinct features on the path
  int32_t path_off;   // first PathNode of the path
  int64_t hist_off;   // 2^depth histogram bins
  int64_t tab_off;    // depth * 2^depth table entries, position-major
  int32_t col_l;      // contraction column of the left (or single) leaf in its class
  int32_t col_r;      // column of the right leaf, -1 for a single
  float w_l, w_r;     // leaf values (w_r = 0 for a single)
};

// A unit of the explain tables: a group's table, or a "quad": the two pair
// groups below the children of one node, merged into one table indexed by
// (path prefix, split at the node, split at its left child, split at its right
// child) with d + 1 values per entry (d = the pairs' depth).  Explain tables
// are indexed by raw splits (bit 1: the row went left), not by whether the row
// follows the path; `mask` holds the path's right turns, so the pattern of a
// raw index r is r ^ mask.  Layout: E = 2^(depth + quad) entries of nv values,
// stored as ceil(nv / 4) float4 planes [plane][slot], value v in component
// v % 4 of plane v / 4 (unused components 0), so that one 16-byte LDS read
// returns four values of an entry; entry I sits at slot
// I ^ (I >> fold_a) ^ (I >> fold_b) of each plane (a bijection), the shifts
// chosen per unit so that the entries rows are likely to read together fall
// in different groups of LDS banks.
struct XUnit {
  int64_t src_l;   // table offset of the (left) group
  int64_t src_r;   // table offset of the right pair group of a quad, -1 otherwise
  int64_t dst;     // offset in the explain tables (floats, multiple of 4)
  int32_t depth;   // depth of the group(s)
  int32_t quad;    // 1 for a quad
  uint32_t mask;   // right turns: all d positions of a group, the d - 2 prefix positions of a quad
  int32_t nv;      // values per entry: depth + quad
  int32_t fold_a;  // entry I sits at slot I ^ (I >> fold_a) ^ (I >> fold_b) of each plane (0: no term)
  int32_t fold_b;
};

// slot of entry I in a plane of an explain-table unit
constexpr int xunit_slot(const XUnit &u, int I) {
  return I ^ (u.fold_a ? I >> u.fold_a : 0) ^ (u.fold_b ? I >> u.fold_b : 0);
}

// floats of a unit in the explain tables
inline int64_t xunit_floats(const XUnit &u) {
  return 4 * (int64_t)((u.nv + 3) / 4) * ((int64_t)1 << (u.depth + u.quad));
}

// A unit of the specialised interaction tables: one group and one feature i
// at its first path position, with the pair tables of i and each other first
// position (its partners, in path order).  The tables are indexed by the raw
// splits r of the group's path (bit 1: the row went left; the pattern is
// r ^ mask) and stored as planes [plane][slot][width]: 4-wide planes for
// partners 0..3, 4..7 (a last group of three partners takes a 4-wide plane
// with one zero), then one 2- or 1-wide plane for a remaining two or one, so
// that a unit of five partners costs one 16-byte and one 4-byte read.  Entry r
// sits at slot r ^ (r >> 3) ^ (r >> 6) of every plane (a bijection on d bits),
// which spreads entries sharing their low three bits (one group of LDS banks
// for 16-byte rows) over all groups.
struct IvUnit {
  int64_t src;     // the group's pair tables (interaction-table offset)
  int64_t dst;     // offset in the interleaved tables (floats, multiple of 4)
  int32_t depth;   // path positions of the group
  int32_t cnt;     // partners, 1..7
  int32_t q[7];    // pair index of (i, partner s) among the group's position pairs
  int32_t group;   // the group
  uint32_t mask;   // right turns of the group's path, root first (MSB)
};

// 4-wide planes of a unit with cnt partners, and the width of its narrow plane (0, 1 or 2)
constexpr int ivunit_quads(int cnt) { return cnt / 4 + (cnt % 4 == 3 ? 1 : 0); }
constexpr int ivunit_tail(int cnt) { return cnt % 4 == 3 ? 0 : cnt % 4; }
// slot of raw index r in every plane
constexpr uint32_t ivunit_slot(uint32_t r) { return r ^ (r >> 3) ^ (r >> 6); }

// floats of a unit in the interleaved interaction tables (a multiple of 4)
constexpr int64_t ivunit_floats(const IvUnit &u) {
  return (((int64_t)(4 * ivunit_quads(u.cnt) + ivunit_tail(u.cnt)) << u.depth) + 3) & ~(int64_t)3;
}

}  // namespace wdf
