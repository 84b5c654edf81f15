// Host-side mesh processing: edges, conductor maps, the structural CSR
// pattern of the A-V matrix, the W pattern, and the scatter lists that let
// the GPU assemble every matrix entry as a fixed-order sum of element values
// (no atomics).  Also the block-Jacobi partition (recursive coordinate
// bisection).  Pure integer/geometry work; all numerics run on the GPU.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.h"

namespace eddy {
namespace {

template <class F>
void parallel_chunks(int64_t n, F&& fn) {
  unsigned hc = std::thread::hardware_concurrency();
  int nth = (int)std::min<unsigned>(hc ? hc : 4, 16);
  if (n < 4096) nth = 1;
  std::vector<std::thread> th;
  int64_t chunk = (n + nth - 1) / nth;
  for (int i = 0; i < nth; ++i) {
    int64_t b = i * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&fn, i, b, e] { fn(i, b, e); });
  }
  for (auto& t : th) t.join();
}

// Stable counting sort of `keys` (0..nkeys-1): returns ptr[nkeys+1] and the
// positions of the items grouped by key, in increasing item order per key.
void group_by(const std::vector<int32_t>& keys, int64_t nkeys, std::vector<int32_t>& ptr,
              std::vector<int32_t>& items) {
  ptr.assign(nkeys + 1, 0);
  for (int32_t k : keys) ptr[k + 1]++;
  for (int64_t i = 0; i < nkeys; ++i) ptr[i + 1] += ptr[i];
  items.resize(keys.size());
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (size_t i = 0; i < keys.size(); ++i) items[fill[keys[i]]++] = (int32_t)i;
}

// Build one CSR structure from per-row (col, contribution) lists produced by
// `gen(row, out)`; entries keep insertion order within equal columns.
template <class Gen>
void build_rows(int64_t nrows, Gen&& gen, std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                std::vector<int32_t>& cptr, std::vector<int32_t>& clist) {
  struct Part {
    std::vector<int32_t> rowlen, col, clen, clist;
  };
  unsigned hc = std::thread::hardware_concurrency();
  int nth = (int)std::min<unsigned>(hc ? hc : 4, 16);
  std::vector<Part> parts(nth);
  int64_t chunk = (nrows + nth - 1) / nth;
  std::vector<std::thread> th;
  for (int i = 0; i < nth; ++i) {
    int64_t b = i * chunk, e = std::min(nrows, b + chunk);
    th.emplace_back([&, i, b, e] {
      Part& P = parts[i];
      std::vector<std::pair<int32_t, int32_t>> buf;
      std::vector<int32_t> ord;
      for (int64_t r = b; r < e; ++r) {
        buf.clear();
        gen(r, buf);
        ord.resize(buf.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return buf[a].first < buf[c].first; });
        int32_t len = 0;
        for (size_t k = 0; k < ord.size(); ++k) {
          const auto& pr = buf[ord[k]];
          if (k == 0 || pr.first != buf[ord[k - 1]].first) {
            P.col.push_back(pr.first);
            P.clen.push_back(0);
            ++len;
          }
          P.clen.back()++;
          P.clist.push_back(pr.second);
        }
        P.rowlen.push_back(len);
      }
    });
  }
  for (auto& t : th) t.join();
  rowptr.assign(nrows + 1, 0);
  int64_t r = 0, nnz = 0, nc = 0;
  for (auto& P : parts) {
    for (int32_t l : P.rowlen) {
      rowptr[r + 1] = rowptr[r] + l;
      ++r;
    }
    nnz += P.col.size();
    nc += P.clist.size();
  }
  col.resize(nnz);
  cptr.assign(nnz + 1, 0);
  clist.resize(nc);
  int64_t oc = 0, ol = 0, oe = 0;
  for (auto& P : parts) {
    std::copy(P.col.begin(), P.col.end(), col.begin() + oc);
    for (size_t k = 0; k < P.clen.size(); ++k) cptr[oe + k + 1] = P.clen[k];
    std::copy(P.clist.begin(), P.clist.end(), clist.begin() + ol);
    oc += P.col.size();
    oe += P.clen.size();
    ol += P.clist.size();
  }
  for (int64_t k = 0; k < nnz; ++k) cptr[k + 1] += cptr[k];
}

int find_root(std::vector<int32_t>& p, int32_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

}  // namespace

// Sliced ELL layout of the CSR pattern (see internal.h).  Sorting by length
// inside a window keeps the padding small (rows of an edge matrix have a few
// distinct lengths) while the row permutation stays local.  Inside a window
// the rows that can hold complex values (V rows and the rows that couple to
// V: edges of conducting tetrahedra and of impedance triangles) come first,
// so that the other slices hold only real values (the SpMV then reads 4-byte
// values there; which slices are real is decided from the values at
// assembly).
eddy_status build_sell(eddy_mesh* m) {
  const int64_t n = m->ndof(), ne = m->ne;
  const int64_t ns = (n + kSellC - 1) / kSellC;
  std::vector<int32_t> order(ns * kSellC, -1);
  std::vector<uint8_t> cplx(n, 0);
  for (int64_t r = 0; r < n; ++r)
    cplx[r] = r >= ne || (m->rowptr[r + 1] > m->rowptr[r] && *std::max_element(m->col.begin() + m->rowptr[r],
                                                                                m->col.begin() + m->rowptr[r + 1]) >= ne);
  for (int64_t w0 = 0; w0 < n; w0 += kSellWindow) {
    const int64_t w1 = std::min<int64_t>(n, w0 + kSellWindow);
    std::iota(order.begin() + w0, order.begin() + w1, (int32_t)w0);
    std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t a, int32_t b) {
      if (cplx[a] != cplx[b]) return cplx[a] > cplx[b];
      return m->rowptr[a + 1] - m->rowptr[a] > m->rowptr[b + 1] - m->rowptr[b];
    });
  }
  m->sell_ptr.assign(ns + 1, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int l = 0; l < kSellC; ++l) {
      const int32_t r = order[s * kSellC + l];
      if (r >= 0) w = std::max(w, m->rowptr[r + 1] - m->rowptr[r]);
    }
    if ((int64_t)m->sell_ptr[s] + (int64_t)w * kSellC >= (int64_t)INT32_MAX) {
      set_error("matrix too large for 32-bit sliced-ELL offsets");
      return EDDY_ERR_ARG;
    }
    m->sell_ptr[s + 1] = m->sell_ptr[s] + w * kSellC;
  }
  const int64_t tot = m->sell_ptr[ns];
  m->sell_row = order;
  m->sell_col.assign(tot, 0);
  m->sell_src.assign(tot, -1);
  parallel_chunks(ns, [&](int, int64_t s0, int64_t s1) {
    for (int64_t s = s0; s < s1; ++s) {
      const int32_t w = (m->sell_ptr[s + 1] - m->sell_ptr[s]) / kSellC;
      for (int l = 0; l < kSellC; ++l) {
        const int32_t r = order[s * kSellC + l];
        const int32_t len = r >= 0 ? m->rowptr[r + 1] - m->rowptr[r] : 0;
        for (int32_t j = 0; j < w; ++j) {
          const int64_t q = m->sell_ptr[s] + (int64_t)j * kSellC + l;
          if (j < len) {
            m->sell_src[q] = m->rowptr[r] + j;
            m->sell_col[q] = m->col[m->rowptr[r] + j];
          } else {
            m->sell_col[q] = r >= 0 ? r : 0;
          }
        }
      }
    }
  });
  return EDDY_OK;
}

eddy_status build_mesh(eddy_mesh* m) {
  const int64_t nv = m->nv, nt = m->nt;
  const int32_t* T = m->tet.data();
  // ---- validation
  for (int64_t i = 0; i < nt * 4; ++i)
    if (T[i] < 0 || T[i] >= nv) { set_error("tet node index out of range"); return EDDY_ERR_ARG; }
  for (int64_t t = 0; t < nt; ++t)
    if (m->region[t] < 0 || m->region[t] >= m->nreg) { set_error("region id out of range"); return EDDY_ERR_ARG; }
  {
    std::atomic<int64_t> bad{-1};
    parallel_chunks(nt, [&](int, int64_t b, int64_t e) {
      for (int64_t t = b; t < e; ++t) {
        const double* p[4];
        for (int k = 0; k < 4; ++k) p[k] = &m->xyz[3 * (int64_t)T[4 * t + k]];
        double E[3][3], L = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) E[i][j] = p[i + 1][j] - p[0][j];
        for (auto& le : kLocalEdge) {
          double d2 = 0;
          for (int j = 0; j < 3; ++j) d2 += (p[le[1]][j] - p[le[0]][j]) * (p[le[1]][j] - p[le[0]][j]);
          L = std::max(L, d2);
        }
        double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                     E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                     E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
        if (!(std::fabs(det) > 1e-12 * L * std::sqrt(L))) bad = t;
      }
    });
    if (bad.load() >= 0) { set_error("degenerate tetrahedron " + std::to_string(bad.load())); return EDDY_ERR_MESH; }
  }
  // ---- impedance-boundary triangles: node ids increasing, conducting region
  const int64_t nf = m->nf;
  for (int64_t f = 0; f < nf; ++f) {
    int32_t* fn = &m->face[3 * f];
    for (int k = 0; k < 3; ++k)
      if (fn[k] < 0 || fn[k] >= nv) { set_error("face node index out of range"); return EDDY_ERR_ARG; }
    std::sort(fn, fn + 3);
    if (fn[0] == fn[1] || fn[1] == fn[2]) { set_error("degenerate face " + std::to_string(f)); return EDDY_ERR_MESH; }
    const int32_t r = m->face_region[f];
    if (r < 0 || r >= m->nreg || !m->is_cond[r]) {
      set_error("face region out of range or not flagged conducting (face " + std::to_string(f) + ")");
      return EDDY_ERR_ARG;
    }
  }
  // ---- edges: group local edges by their low node, sort each group by the high node
  std::vector<int32_t> lo(nt * 6), hi(nt * 6);
  m->signbits.assign(nt, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int l = 0; l < 6; ++l) {
      int32_t a = T[4 * t + kLocalEdge[l][0]], b = T[4 * t + kLocalEdge[l][1]];
      lo[6 * t + l] = std::min(a, b);
      hi[6 * t + l] = std::max(a, b);
      if (a > b) m->signbits[t] |= (uint8_t)(1u << l);
    }
  std::vector<int32_t> bptr, occ;
  group_by(lo, nv, bptr, occ);
  m->tet2edge.assign(nt * 6, -1);
  m->edges.clear();
  {
    std::vector<int32_t> tmp;
    int32_t eid = 0;
    for (int64_t a = 0; a < nv; ++a) {
      tmp.assign(occ.begin() + bptr[a], occ.begin() + bptr[a + 1]);
      std::stable_sort(tmp.begin(), tmp.end(), [&](int32_t x, int32_t y) { return hi[x] < hi[y]; });
      for (size_t k = 0; k < tmp.size(); ++k) {
        if (k == 0 || hi[tmp[k]] != hi[tmp[k - 1]]) {
          m->edges.push_back((int32_t)a);
          m->edges.push_back(hi[tmp[k]]);
          ++eid;
        }
        m->tet2edge[tmp[k]] = eid - 1;
      }
    }
    m->ne = eid;
  }
  const int64_t ne = m->ne;
  // local edges (0,1), (0,2), (1,2) of each face: edges are numbered by low
  // node, then high node, so a binary search inside the low node's run
  {
    std::vector<int32_t> first(nv + 1, 0);
    for (int64_t e = 0; e < ne; ++e) first[m->edges[2 * e] + 1]++;
    for (int64_t a = 0; a < nv; ++a) first[a + 1] += first[a];
    m->face2edge.assign(nf * 3, -1);
    constexpr int fa[3] = {0, 0, 1}, fb[3] = {1, 2, 2};
    for (int64_t f = 0; f < nf; ++f)
      for (int l = 0; l < 3; ++l) {
        const int32_t a = m->face[3 * f + fa[l]], b = m->face[3 * f + fb[l]];
        int32_t lo = first[a], hi = first[a + 1];
        while (lo < hi) {
          const int32_t mid = (lo + hi) / 2;
          if (m->edges[2 * mid + 1] < b) lo = mid + 1;
          else hi = mid;
        }
        if (lo >= first[a + 1] || m->edges[2 * lo + 1] != b) {
          set_error("an edge of face " + std::to_string(f) + " is not an edge of the tetrahedra");
          return EDDY_ERR_MESH;
        }
        m->face2edge[3 * f + l] = lo;
      }
  }
  // ---- conductor maps
  m->cidx.assign(nt, -1);
  m->vmap.assign(nv, -1);
  int64_t nct = 0;
  for (int64_t t = 0; t < nt; ++t)
    if (m->is_cond[m->region[t]]) {
      m->cidx[t] = (int32_t)nct++;
      for (int k = 0; k < 4; ++k) m->vmap[T[4 * t + k]] = 0;
    }
  for (int64_t i = 0; i < nf * 3; ++i) m->vmap[m->face[i]] = 0;     // V on impedance surfaces
  m->nct = nct;
  m->cond_nodes.clear();
  for (int64_t n = 0; n < nv; ++n)
    if (m->vmap[n] == 0) {
      m->vmap[n] = (int32_t)m->cond_nodes.size();
      m->cond_nodes.push_back((int32_t)n);
    }
  m->nc = (int64_t)m->cond_nodes.size();
  const int64_t nc = m->nc;
  // conductor components (union-find over conducting tetrahedra)
  {
    std::vector<int32_t> par(nc);
    std::iota(par.begin(), par.end(), 0);
    for (int64_t t = 0; t < nt; ++t)
      if (m->cidx[t] >= 0) {
        int32_t r0 = find_root(par, m->vmap[T[4 * t]]);
        for (int k = 1; k < 4; ++k) {
          int32_t rk = find_root(par, m->vmap[T[4 * t + k]]);
          if (rk != r0) par[std::max(rk, r0)] = std::min(rk, r0), r0 = std::min(rk, r0);
        }
      }
    for (int64_t f = 0; f < nf; ++f) {
      int32_t r0 = find_root(par, m->vmap[m->face[3 * f]]);
      for (int k = 1; k < 3; ++k) {
        int32_t rk = find_root(par, m->vmap[m->face[3 * f + k]]);
        if (rk != r0) par[std::max(rk, r0)] = std::min(rk, r0), r0 = std::min(rk, r0);
      }
    }
    m->comp.assign(nc, -1);
    std::vector<int32_t> label(nc, -1);
    int32_t nl = 0;
    for (int64_t i = 0; i < nc; ++i) {
      int32_t r = find_root(par, (int32_t)i);
      if (label[r] < 0) label[r] = nl++;
      m->comp[i] = label[r];
    }
    m->ncomp = nl;
  }
  m->edge_v.assign(ne * 2, -1);
  for (int64_t t = 0; t < nt; ++t)
    if (m->cidx[t] >= 0)
      for (int l = 0; l < 6; ++l) {
        int32_t e = m->tet2edge[6 * t + l];
        m->edge_v[2 * e] = m->vmap[m->edges[2 * e]];
        m->edge_v[2 * e + 1] = m->vmap[m->edges[2 * e + 1]];
      }
  // ---- incidences: edge -> (t, l) occurrences; conductor node -> (t, k) in conducting tets
  std::vector<int32_t> eptr, eocc;
  group_by(m->tet2edge, ne, eptr, eocc);
  std::vector<int32_t> vkeys;
  std::vector<int32_t> vsrc;
  vkeys.reserve(nct * 4);
  vsrc.reserve(nct * 4);
  for (int64_t t = 0; t < nt; ++t)
    if (m->cidx[t] >= 0)
      for (int k = 0; k < 4; ++k) {
        vkeys.push_back(m->vmap[T[4 * t + k]]);
        vsrc.push_back((int32_t)(4 * t + k));
      }
  std::vector<int32_t> vptr, vitem;
  group_by(vkeys, nc, vptr, vitem);
  for (auto& x : vitem) x = vsrc[x];   // -> 4*t + k, increasing t per node
  // face occurrences: edge -> 3*f + l, V node -> 3*f + k (increasing f)
  std::vector<int32_t> feptr, feocc, fvptr, fvocc;
  group_by(m->face2edge, ne, feptr, feocc);
  {
    std::vector<int32_t> fv(nf * 3);
    for (int64_t i = 0; i < nf * 3; ++i) fv[i] = m->vmap[m->face[i]];
    group_by(fv, nc, fvptr, fvocc);
  }
  // ---- M pattern + scatter lists (slots: tetrahedra AA, AV, VV, then faces AA, AV, VV)
  const int64_t AV0 = 21 * nt, VV0 = 21 * nt + 24 * nct;
  const int64_t FA0 = 21 * nt + 34 * nct, FAV0 = FA0 + 6 * nf, FVV0 = FAV0 + 9 * nf;
  auto genM = [&](int64_t r, std::vector<std::pair<int32_t, int32_t>>& out) {
    if (r < ne) {
      for (int32_t p = eptr[r]; p < eptr[r + 1]; ++p) {
        int64_t o = eocc[p], t = o / 6;
        int l = (int)(o % 6);
        for (int mm = 0; mm < 6; ++mm)
          out.emplace_back(m->tet2edge[6 * t + mm], (int32_t)(pair6(l, mm) * nt + t));
        int32_t c = m->cidx[t];
        if (c >= 0)
          for (int k = 0; k < 4; ++k)
            out.emplace_back((int32_t)(ne + m->vmap[T[4 * t + k]]), (int32_t)(AV0 + (l * 4 + k) * nct + c));
      }
      for (int32_t p = feptr[r]; p < feptr[r + 1]; ++p) {
        const int64_t f = feocc[p] / 3;
        const int l = feocc[p] % 3;
        for (int mm = 0; mm < 3; ++mm)
          out.emplace_back(m->face2edge[3 * f + mm], (int32_t)(FA0 + pair3(l, mm) * nf + f));
        for (int k = 0; k < 3; ++k)
          out.emplace_back((int32_t)(ne + m->vmap[m->face[3 * f + k]]), (int32_t)(FAV0 + (l * 3 + k) * nf + f));
      }
    } else {
      int64_t n = r - ne;
      for (int32_t p = vptr[n]; p < vptr[n + 1]; ++p) {
        int64_t o = vitem[p], t = o / 4;
        int k = (int)(o % 4);
        int32_t c = m->cidx[t];
        for (int mm = 0; mm < 6; ++mm)
          out.emplace_back(m->tet2edge[6 * t + mm], (int32_t)(AV0 + (mm * 4 + k) * nct + c));
        for (int kk = 0; kk < 4; ++kk)
          out.emplace_back((int32_t)(ne + m->vmap[T[4 * t + kk]]), (int32_t)(VV0 + pair4(k, kk) * nct + c));
      }
      for (int32_t p = fvptr[n]; p < fvptr[n + 1]; ++p) {
        const int64_t f = fvocc[p] / 3;
        const int k = fvocc[p] % 3;
        for (int mm = 0; mm < 3; ++mm)
          out.emplace_back(m->face2edge[3 * f + mm], (int32_t)(FAV0 + (mm * 3 + k) * nf + f));
        for (int kk = 0; kk < 3; ++kk)
          out.emplace_back((int32_t)(ne + m->vmap[m->face[3 * f + kk]]), (int32_t)(FVV0 + pair3(k, kk) * nf + f));
      }
    }
  };
  if (21 * nt + 34 * nct + 21 * nf >= (int64_t)INT32_MAX || 24 * nt >= (int64_t)INT32_MAX ||
      nt + nf >= (int64_t)INT32_MAX) {
    set_error("mesh too large for 32-bit scatter indices");
    return EDDY_ERR_ARG;
  }
  build_rows(ne + nc, genM, m->rowptr, m->col, m->cptr, m->clist);
  if ((int64_t)m->clist.size() >= (int64_t)INT32_MAX) { set_error("too many contributions"); return EDDY_ERR_ARG; }
  m->diagpos.assign(ne + nc, -1);
  for (int64_t r = 0; r < ne + nc; ++r)
    for (int32_t p = m->rowptr[r]; p < m->rowptr[r + 1]; ++p)
      if (m->col[p] == r) m->diagpos[r] = p;
  for (int64_t r = 0; r < ne + nc; ++r)
    if (m->diagpos[r] < 0) { set_error("row without a diagonal entry"); return EDDY_ERR_MESH; }
  if (eddy_status st = build_sell(m); st != EDDY_OK) return st;
  // ---- W pattern + scatter lists
  auto genW = [&](int64_t r, std::vector<std::pair<int32_t, int32_t>>& out) {
    for (int32_t p = eptr[r]; p < eptr[r + 1]; ++p) {
      int64_t o = eocc[p], t = o / 6;
      int l = (int)(o % 6);
      for (int k = 0; k < 4; ++k) out.emplace_back(T[4 * t + k], (int32_t)((l * 4 + k) * nt + t));
    }
  };
  build_rows(ne, genW, m->wrowptr, m->wcol, m->wcptr, m->wclist);
  for (int64_t r = 0; r < ne; ++r)
    if (m->wrowptr[r + 1] - m->wrowptr[r] > kMaxWRow) {
      set_error("an edge touches more than " + std::to_string(kMaxWRow) + " nodes through its tetrahedra");
      return EDDY_ERR_MESH;
    }
  group_by(m->wcol, nv, m->wtrowptr, m->wtperm);
  m->wtcol.resize(m->wcol.size());
  {
    std::vector<int32_t> rowof(m->wcol.size());
    for (int64_t r = 0; r < ne; ++r)
      for (int32_t p = m->wrowptr[r]; p < m->wrowptr[r + 1]; ++p) rowof[p] = (int32_t)r;
    for (size_t q = 0; q < m->wtperm.size(); ++q) m->wtcol[q] = rowof[m->wtperm[q]];
  }
  // ---- pattern of L = W^T G: row n couples the endpoints of the edges in row n of W^T
  {
    m->lrowptr.assign(nv + 1, 0);
    std::vector<std::vector<int32_t>> rows(nv);
    parallel_chunks(nv, [&](int, int64_t a, int64_t b) {
      for (int64_t n = a; n < b; ++n) {
        auto& r = rows[n];
        for (int32_t q = m->wtrowptr[n]; q < m->wtrowptr[n + 1]; ++q) {
          const int32_t e = m->wtcol[q];
          r.push_back(m->edges[2 * e]);
          r.push_back(m->edges[2 * e + 1]);
        }
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
      }
    });
    for (int64_t n = 0; n < nv; ++n) m->lrowptr[n + 1] = m->lrowptr[n] + (int32_t)rows[n].size();
    m->lcol.resize(m->lrowptr[nv]);
    for (int64_t n = 0; n < nv; ++n) std::copy(rows[n].begin(), rows[n].end(), m->lcol.begin() + m->lrowptr[n]);
  }
  // ---- D0 (all tets), lumped conductor mass (conducting tets), rhs gathers
  {
    std::vector<int32_t> item;
    group_by(m->tet, nv, m->d0ptr, item);
    m->d0list.resize(item.size());
    for (size_t i = 0; i < item.size(); ++i) m->d0list[i] = item[i] / 4;
    // lumped V-node weights: |K|/4 of conducting tets (vol4[t]), then
    // |T|/3 of impedance triangles (vol4[nt + f])
    m->lcptr.assign(nc + 1, 0);
    m->lclist.clear();
    m->lclist.reserve(vitem.size() + fvocc.size());
    for (int64_t n = 0; n < nc; ++n) {
      for (int32_t p = vptr[n]; p < vptr[n + 1]; ++p) m->lclist.push_back(vitem[p] / 4);
      for (int32_t p = fvptr[n]; p < fvptr[n + 1]; ++p) m->lclist.push_back((int32_t)(nt + fvocc[p] / 3));
      m->lcptr[n + 1] = (int32_t)m->lclist.size();
    }
    m->rptr = eptr;
    m->rlist.resize(eocc.size());
    for (size_t i = 0; i < eocc.size(); ++i) {
      int64_t o = eocc[i];
      m->rlist[i] = (int32_t)((o % 6) * nt + o / 6);
    }
  }
  return EDDY_OK;
}

// Recursive coordinate bisection of the DOF positions (edge midpoints, then
// conductor nodes).  A set S (sorted by DOF id) with nb = ceil(|S|/b) <= 1 is
// a block; otherwise it is split along the axis of largest extent (lowest
// axis on ties) after sorting by (coordinate, id), the left part receiving
// floor(|S| * floor(nb/2) / nb) DOFs.  Blocks are emitted depth-first, left
// first; DOFs inside a block are in increasing id.
eddy_status build_blocks(eddy_mesh* m, int32_t b) {
  if (m->blk_b == b) return EDDY_OK;
  const int64_t n = m->ndof(), ne = m->ne;
  std::vector<double> X(n * 3);
  for (int64_t e = 0; e < ne; ++e)
    for (int j = 0; j < 3; ++j)
      X[3 * e + j] = (m->xyz[3 * (int64_t)m->edges[2 * e] + j] + m->xyz[3 * (int64_t)m->edges[2 * e + 1] + j]) * 0.5;
  for (int64_t c = 0; c < m->nc; ++c)
    for (int j = 0; j < 3; ++j) X[3 * (ne + c) + j] = m->xyz[3 * (int64_t)m->cond_nodes[c] + j];
  std::vector<int32_t> ids(n);
  std::iota(ids.begin(), ids.end(), 0);
  m->blk_ptr.assign(1, 0);
  m->blk_dofs.clear();
  m->blk_dofs.reserve(n);
  struct Range { int64_t b, e; };
  std::vector<Range> stack{{0, n}};
  while (!stack.empty()) {
    Range R = stack.back();
    stack.pop_back();
    int64_t sz = R.e - R.b;
    int64_t nb = (sz + b - 1) / b;
    if (nb <= 1) {
      m->blk_dofs.insert(m->blk_dofs.end(), ids.begin() + R.b, ids.begin() + R.e);
      m->blk_ptr.push_back((int32_t)m->blk_dofs.size());
      continue;
    }
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = R.b; i < R.e; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = X[3 * (int64_t)ids[i] + j];
        mn[j] = std::min(mn[j], v);
        mx[j] = std::max(mx[j], v);
      }
    int ax = 0;
    double best = mx[0] - mn[0];
    for (int j = 1; j < 3; ++j)
      if (mx[j] - mn[j] > best) best = mx[j] - mn[j], ax = j;
    auto first = ids.begin() + R.b, last = ids.begin() + R.e;
    std::sort(first, last, [&](int32_t a, int32_t c) {
      double xa = X[3 * (int64_t)a + ax], xc = X[3 * (int64_t)c + ax];
      return xa < xc || (xa == xc && a < c);
    });
    int64_t s = (sz * (nb / 2)) / nb;
    std::sort(first, first + s);
    std::sort(first + s, last);
    stack.push_back({R.b + s, R.e});
    stack.push_back({R.b, R.b + s});
  }
  m->blk_b = b;
  return EDDY_OK;
}

eddy_status build_subdomains(eddy_mesh* m, int32_t b, std::vector<int32_t>& sub_ptr,
                             std::vector<int32_t>& sub_of_dof, std::vector<int32_t>& adj,
                             std::vector<uint32_t>& regmask) {
  if (eddy_status st = build_blocks(m, b); st != EDDY_OK) return st;
  if (m->nreg > 32) { set_error("the learned correction supports at most 32 regions"); return EDDY_ERR_ARG; }
  const int64_t n = m->ndof(), nb = (int64_t)m->blk_ptr.size() - 1;
  sub_ptr.assign(kGnnP + 1, 0);
  sub_of_dof.assign(n, 0);
  for (int p = 0; p <= kGnnP; ++p) {
    const int64_t k0 = (p * nb + kGnnP - 1) / kGnnP;   // first block with floor(k P / nb) >= p
    sub_ptr[p] = m->blk_ptr[std::min<int64_t>(k0, nb)];
  }
  for (int64_t k = 0; k < nb; ++k)
    for (int32_t q = m->blk_ptr[k]; q < m->blk_ptr[k + 1]; ++q) sub_of_dof[m->blk_dofs[q]] = (int32_t)((k * kGnnP) / nb);
  adj.assign(kGnnP * kGnnP, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int32_t p = m->rowptr[r]; p < m->rowptr[r + 1]; ++p) {
      const int32_t a = sub_of_dof[r], c = sub_of_dof[m->col[p]];
      if (a != c) adj[a * kGnnP + c] = 1;
    }
  regmask.assign(n, 0u);
  for (int64_t t = 0; t < m->nt; ++t) {
    const uint32_t bit = 1u << m->region[t];
    for (int l = 0; l < 6; ++l) regmask[m->tet2edge[6 * t + l]] |= bit;
    for (int k = 0; k < 4; ++k) {
      const int32_t c = m->vmap[m->tet[4 * t + k]];
      if (c >= 0) regmask[m->ne + c] |= bit;
    }
  }
  return EDDY_OK;
}

}  // namespace eddy

// ---- impedance boundary: remove the tetrahedra of the flagged regions and
// return their interface with the rest as surface triangles (Section 2,
// Eqs. 8-10).  Faces are sorted node triples; the interface is the set of
// faces of removed tetrahedra that are also faces of kept ones.
extern "C" eddy_status eddy_ibc_split(int64_t nv, const double* xyz, int64_t nt, const int32_t* tet,
                                      const int32_t* region, int32_t nreg, const int32_t* is_ibc, int64_t* nv_out,
                                      int64_t* nt_out, int64_t* nf_out, double* xyz_out, int32_t* tet_out,
                                      int32_t* region_out, int32_t* face_out, int32_t* face_region_out,
                                      int32_t* node_map) {
  using namespace eddy;
  if (!xyz || !tet || !region || !is_ibc || !nv_out || !nt_out || !nf_out) {
    set_error("NULL argument");
    return EDDY_ERR_ARG;
  }
  if (nv < 1 || nt < 1 || nreg < 1 || nv >= INT32_MAX || nt * 4 >= INT32_MAX) {
    set_error("mesh sizes out of range");
    return EDDY_ERR_ARG;
  }
  const bool fill = xyz_out || tet_out || region_out || face_out || face_region_out || node_map;
  if (fill && !(xyz_out && tet_out && region_out && face_out && face_region_out && node_map)) {
    set_error("either all output arrays or none");
    return EDDY_ERR_ARG;
  }
  try {
    for (int64_t i = 0; i < nt * 4; ++i)
      if (tet[i] < 0 || tet[i] >= nv) { set_error("tet node index out of range"); return EDDY_ERR_ARG; }
    for (int64_t t = 0; t < nt; ++t)
      if (region[t] < 0 || region[t] >= nreg) { set_error("region id out of range"); return EDDY_ERR_ARG; }
    struct Face {
      int32_t n[3], reg;
      bool operator<(const Face& o) const {
        return n[0] != o.n[0] ? n[0] < o.n[0] : n[1] != o.n[1] ? n[1] < o.n[1] : n[2] < o.n[2];
      }
      bool same(const Face& o) const { return n[0] == o.n[0] && n[1] == o.n[1] && n[2] == o.n[2]; }
    };
    constexpr int tf[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    std::vector<Face> kept, gone;
    std::vector<char> used(nv, 0);
    int64_t ntk = 0;
    for (int64_t t = 0; t < nt; ++t) {
      const bool g = is_ibc[region[t]] != 0;
      if (!g) {
        ++ntk;
        for (int k = 0; k < 4; ++k) used[tet[4 * t + k]] = 1;
      }
      for (auto& q : tf) {
        Face f;
        for (int k = 0; k < 3; ++k) f.n[k] = tet[4 * t + q[k]];
        std::sort(f.n, f.n + 3);
        f.reg = region[t];
        (g ? gone : kept).push_back(f);
      }
    }
    std::sort(kept.begin(), kept.end());
    std::sort(gone.begin(), gone.end());
    std::vector<Face> iface;
    for (size_t i = 0; i < gone.size(); ++i) {
      if (i > 0 && gone[i].same(gone[i - 1])) continue;
      auto it = std::lower_bound(kept.begin(), kept.end(), gone[i]);
      if (it != kept.end() && it->same(gone[i])) iface.push_back(gone[i]);
    }
    int64_t nvk = 0;
    std::vector<int32_t> map(nv, -1);
    for (int64_t n = 0; n < nv; ++n)
      if (used[n]) map[n] = (int32_t)nvk++;
    *nv_out = nvk;
    *nt_out = ntk;
    *nf_out = (int64_t)iface.size();
    if (!fill) return EDDY_OK;
    std::copy(map.begin(), map.end(), node_map);
    for (int64_t n = 0; n < nv; ++n)
      if (map[n] >= 0)
        for (int j = 0; j < 3; ++j) xyz_out[3 * (int64_t)map[n] + j] = xyz[3 * n + j];
    int64_t o = 0;
    for (int64_t t = 0; t < nt; ++t)
      if (!is_ibc[region[t]]) {
        for (int k = 0; k < 4; ++k) tet_out[4 * o + k] = map[tet[4 * t + k]];
        region_out[o++] = region[t];
      }
    for (size_t f = 0; f < iface.size(); ++f) {
      for (int k = 0; k < 3; ++k) face_out[3 * f + k] = map[iface[f].n[k]];
      face_region_out[f] = iface[f].reg;
    }
  } catch (const std::exception& e) {
    set_error(std::string("host failure: ") + e.what());
    return EDDY_ERR_ARG;
  }
  return EDDY_OK;
}
