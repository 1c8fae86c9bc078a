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

}  // namespace wdf
