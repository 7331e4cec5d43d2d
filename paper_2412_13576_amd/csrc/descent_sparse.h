// Sparse-basis descent (binary32): declarations shared by the host setup in
// extract.cpp and the kernel in descent_sparse.hip.
#pragma once

#include <cstdint>
#include <vector>

#include "graver_internal.h"

namespace graver {

// Row lists of B for the sparse descent, built on the host.  Rows are taken
// in order of decreasing nonzero count and dealt to the 64 lanes of a
// wavefront in slots of 64 rows; every row of a slot is padded to the
// slot's longest row, so the slot structure is the same in every lane.
//   slot[t]             width of slot t | its first entry << 16
//   ent[e * 64 + lane]  entry e of the lane: column | (uint16) B_ij << 16
//                       (padding: column 0, value 0)
//   row[t * 64 + lane]  row of slot t: i | (u_i - l_i) << 16 (0xFFFF: none)
struct SparseImage {
  int ew = 0;  // entries per lane (sum of the slot widths)
  int nc = 0;  // slots, ceil(n / 64); 0: no image
  uint32_t slot[16] = {};
  std::vector<uint32_t> ent, row;
};

// Builds the image of the n x d basis B (row-major, host) with box widths
// u - l.  Returns false when B does not fit the form: n or d > 1024, an
// entry beyond +-32767, or more than 128 row-list entries per lane.
bool sparse_image_build(int n, int d, const int64_t* B, const int64_t* l, const int64_t* u, SparseImage& img);
// Whether the sparse form is expected to beat the matrix-core descent: its
// padded row lists hold at most an eighth of the n x d products.
bool sparse_form_pays(const SparseImage& img, int n, int d);

// One launch: a.T iterations of every start (state in the wave-native
// binary32 layout of the matrix-core kernels with blk16(d) column blocks),
// candidates appended to a.log.  dev_ent / dev_row are the image's arrays
// on the device; rlim is the exact range of the rounded coordinates.
hipError_t launch_descent_sparse(hipStream_t s, const DescentArgs& a, const SparseImage& img, const uint32_t* dev_ent,
                                 const uint32_t* dev_row, float* state, int64_t per, unsigned long long* counters,
                                 float rlim);

}  // namespace graver
