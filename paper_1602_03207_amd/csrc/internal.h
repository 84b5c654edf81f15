// Internal definitions shared by the host mesh code, the API layer and the
// HIP kernels.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "eddy.h"

// ---------------------------------------------------------------------------
// Element-buffer layout: the element kernel writes every element-level value
// exactly once at these positions; the scatter maps built on the host refer
// to them.  Local edges of a tetrahedron are (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
//
//   ebuf (complex):  AA  pair slot p (0..20) of the 6x6 A-A block: p*nt + t
//                    AV  (l*4 + k) of the 6x4 A-V block:           AV0 + (l*4+k)*nct + c
//                    VV  pair slot q (0..9) of the 4x4 V-V block:  VV0 + q*nct + c
//   wbuf (real):     W_e (l*4 + k):                                 (l*4+k)*nt + t
//   vol4 (real):     |K| / 4:                                       t
//   rbuf (real):     int J . w_l:                                   l*nt + t
// with t the tetrahedron, c its compact conductor index (nct of them).
// ---------------------------------------------------------------------------
namespace eddy {

constexpr int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr int kMaxBlock = 64;       // block-Jacobi block size limit (LDS-resident inverse)
constexpr int kMaxRestart = 64;
constexpr int kMaxWRow = 32;       // max nodes adjacent to one edge (LDS-staged gauge blocks)
constexpr int kBatchChunk = 8;     // systems per pass of the batched SpMV / block-Jacobi kernels
constexpr int kMaxDzCols = 4;      // free-configuration solutions per pass of the defect-volume kernel
// Learned coarse correction: a graph network on kGnnP subdomains, kGnnFin
// input features, width kGnnWidth, kGnnFout outputs (the first two used).
// Parameters (float32, in this order, row-major): W0 [Fin x W], b0 [W],
// W1 [W x W], b1, W2 [W x W], b2, W3 [W x Fout], b3 [Fout].
constexpr int kGnnP = 64;
constexpr int kGnnFin = 16;
constexpr int kGnnWidth = 64;
constexpr int kGnnFout = 16;
constexpr int kGnnOffW0 = 0;
constexpr int kGnnOffB0 = kGnnOffW0 + kGnnFin * kGnnWidth;
constexpr int kGnnOffW1 = kGnnOffB0 + kGnnWidth;
constexpr int kGnnOffB1 = kGnnOffW1 + kGnnWidth * kGnnWidth;
constexpr int kGnnOffW2 = kGnnOffB1 + kGnnWidth;
constexpr int kGnnOffB2 = kGnnOffW2 + kGnnWidth * kGnnWidth;
constexpr int kGnnOffW3 = kGnnOffB2 + kGnnWidth;
constexpr int kGnnOffB3 = kGnnOffW3 + kGnnWidth * kGnnFout;
constexpr int kGnnParams = kGnnOffB3 + kGnnFout;
// per-sample scratch of the network kernels (float32 words): 7 float32
// [P x W] arrays, Y [P x Fout], and bf16 arrays (2 per word): Xb [P x Fin],
// 6 of [P x W], dYb [P x Fout]
constexpr int kGnnScratch = 7 * kGnnP * kGnnWidth + kGnnP * kGnnFout +
                            (kGnnP * kGnnFin + 6 * kGnnP * kGnnWidth + kGnnP * kGnnFout) / 2;
// Sliced ELL copy of M for the SpMV: slices of kSellC rows (one wavefront,
// one lane per row), rows sorted by decreasing length inside windows of
// kSellWindow rows; slice s holds its width x kSellC entries column-major.
constexpr int kSellC = 64;
constexpr int kSellWindow = 1024;

// Krylov basis entry in complex half precision (real part in the low 16
// bits), stored scaled by 2^14: the basis vectors have unit norm, so every
// entry is at most 1 in magnitude and the scaled parts stay inside
// binary16's normal range down to ~4e-9.
struct hbasis {
  uint32_t b;
};

inline int pair6(int l, int m) {    // upper-triangle slot of a symmetric 6x6
  if (l > m) { int t = l; l = m; m = t; }
  return l * 6 - (l * (l - 1)) / 2 + (m - l);
}
inline int pair3(int i, int j) {    // upper-triangle slot of a symmetric 3x3
  if (i > j) { int t = i; i = j; j = t; }
  return i == 0 ? j : (i == 1 ? 2 + j : 5);
}
inline int pair4(int i, int j) {    // upper-triangle slot of a symmetric 4x4
  if (i > j) { int t = i; i = j; j = t; }
  return i * 4 - (i * (i - 1)) / 2 + (j - i);
}

void set_error(const std::string& msg);

}  // namespace eddy

struct eddy_mesh {
  int64_t nv = 0, nt = 0;
  int32_t nreg = 0;
  std::vector<double> xyz;          // nv*3
  std::vector<int32_t> tet;         // nt*4
  std::vector<int32_t> region;      // nt
  std::vector<int32_t> is_cond;     // nreg
  // impedance-boundary triangles (surface conductors, Eqs. 8-10): node ids
  // increasing per triangle, the region whose sigma and nu give 1/Z, and the
  // edges of the local pairs (0,1), (0,2), (1,2)
  int64_t nf = 0;
  std::vector<int32_t> face, face_region, face2edge;
  uint64_t geom_hash = 0;           // FNV-1a over xyz, tet, region and faces (same geometry <=> same hash)
  // topology
  int64_t ne = 0, nc = 0, nct = 0;
  int32_t ncomp = 0;
  std::vector<int32_t> edges;       // ne*2 (lo, hi)
  std::vector<int32_t> tet2edge;    // nt*6
  std::vector<uint8_t> signbits;    // nt; bit l set if local edge l runs hi -> lo
  std::vector<int32_t> cidx;        // nt; compact conductor index or -1
  std::vector<int32_t> cond_nodes;  // nc
  std::vector<int32_t> vmap;        // nv; conductor index or -1
  std::vector<int32_t> comp;        // nc; conductor component
  std::vector<int32_t> edge_v;      // ne*2; conductor ids of (lo, hi) on conducting edges, else -1
  // M: structural CSR pattern and scatter lists into ebuf
  std::vector<int32_t> rowptr, col, diagpos, cptr, clist;
  // W (ne x nv): pattern and scatter lists into wbuf; W^T via a permutation
  std::vector<int32_t> wrowptr, wcol, wcptr, wclist;
  std::vector<int32_t> wtrowptr, wtcol, wtperm;
  // L = W^T G (nodal, symmetric; the Coulomb projection's operator): pattern
  std::vector<int32_t> lrowptr, lcol;
  // gathers of vol4 (D0 over all tets, lumped conductor mass) and of rbuf
  std::vector<int32_t> d0ptr, d0list, lcptr, lclist, rptr, rlist;
  // sliced ELL: sell_ptr[nslices+1] (entry offsets), sell_row[nslices*kSellC]
  // (row of each lane, -1 past the end), sell_col / sell_src per entry (CSR
  // position of the value, -1 for padding, whose column is the lane's row)
  std::vector<int32_t> sell_ptr, sell_row, sell_col, sell_src;
  // cached block partition
  int32_t blk_b = 0;
  std::vector<int32_t> blk_ptr, blk_dofs;

  int64_t ndof() const { return ne + nc; }
  int64_t nnz() const { return (int64_t)col.size(); }
  int64_t nnzw() const { return (int64_t)wcol.size(); }
};

namespace eddy {
eddy_status build_mesh(eddy_mesh* m);                  // topology + patterns + maps
eddy_status build_blocks(eddy_mesh* m, int32_t b);     // RCB partition (cached)
// Subdomains of the learned correction: the blocks of size b (bisection
// order) grouped into kGnnP runs of equal block count.  sub_ptr[kGnnP + 1]:
// ranges in the block DOF list; sub_of_dof[ndof]; adj[kGnnP * kGnnP]: 1 where
// M couples two different subdomains; regmask[ndof]: bit r set if a
// tetrahedron of region r contains the DOF (edge, or conductor node).
eddy_status build_subdomains(eddy_mesh* m, int32_t b, std::vector<int32_t>& sub_ptr,
                             std::vector<int32_t>& sub_of_dof, std::vector<int32_t>& adj,
                             std::vector<uint32_t>& regmask);
}  // namespace eddy
