// Host-side topology, decomposition and point location (see host_mesh.h).
#include "host_mesh.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>

namespace mx {

namespace {

const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int LF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
// local edge index of the face edges (0,1), (0,2), (1,2) of each local face
const int FE[4][3] = {{0, 1, 3}, {0, 2, 4}, {1, 2, 5}, {3, 4, 5}};

struct FaceKey {
  uint64_t ab;
  uint32_t c;
  uint32_t occ;  // tet*4 + local face
};

// counting sort of (key -> item) pairs, items in ascending item order per key
void bucket(int64_t nkeys, const std::vector<int32_t>& keys, int per_item,
            std::vector<int64_t>& ptr, std::vector<int32_t>& out) {
  ptr.assign(nkeys + 1, 0);
  for (int32_t k : keys) ptr[k + 1]++;
  for (int64_t i = 0; i < nkeys; ++i) ptr[i + 1] += ptr[i];
  out.resize(keys.size());
  std::vector<int64_t> cur(ptr.begin(), ptr.end() - 1);
  for (size_t j = 0; j < keys.size(); ++j) out[cur[keys[j]]++] = (int32_t)(j / per_item);
}

}  // namespace

std::string build_topology(int32_t nv, int32_t nt, const double* xyz, const int32_t* tet,
                           Topology& T) {
  if (nv <= 0 || nt <= 0 || !xyz || !tet) return "empty mesh";
  T = Topology();
  T.nv = nv;
  T.nt = nt;
  T.xyz.assign(xyz, xyz + 3 * (size_t)nv);
  T.tet_in.assign(tet, tet + 4 * (size_t)nt);
  for (size_t i = 0; i < T.xyz.size(); ++i)
    if (!std::isfinite(T.xyz[i])) return "non-finite vertex coordinate";
  T.ts.resize(4 * (size_t)nt);
  for (int32_t t = 0; t < nt; ++t) {
    int32_t v[4];
    for (int k = 0; k < 4; ++k) {
      v[k] = tet[4 * (size_t)t + k];
      if (v[k] < 0 || v[k] >= nv) return "tetrahedron vertex id out of range";
    }
    std::sort(v, v + 4);
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) return "tetrahedron with repeated vertex";
    const double* p0 = &xyz[3 * (size_t)v[0]];
    double d[3][3];
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) d[k][c] = xyz[3 * (size_t)v[k + 1] + c] - p0[c];
    double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                 d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                 d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    if (!(std::fabs(det) > 0.0)) return "degenerate (zero-volume) tetrahedron";
    for (int k = 0; k < 4; ++k) T.ts[4 * (size_t)t + k] = v[k];
  }
  const uint64_t unv = (uint64_t)nv;
  // ---- edges
  std::vector<uint64_t> ek(6 * (size_t)nt);
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < nt; ++t)
    for (int le = 0; le < 6; ++le)
      ek[6 * (size_t)t + le] = (uint64_t)T.ts[4 * (size_t)t + LE[le][0]] * unv +
                               (uint64_t)T.ts[4 * (size_t)t + LE[le][1]];
  std::vector<uint64_t> uk(ek);
  std::sort(uk.begin(), uk.end());
  uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
  T.ne = (int64_t)uk.size();
  if (T.ne >= (int64_t)INT32_MAX) return "too many edges";
  T.edges.resize(2 * (size_t)T.ne);
  for (int64_t e = 0; e < T.ne; ++e) {
    T.edges[2 * e] = (int32_t)(uk[e] / unv);
    T.edges[2 * e + 1] = (int32_t)(uk[e] % unv);
  }
  T.t2e.resize(6 * (size_t)nt);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < 6 * (int64_t)nt; ++j)
    T.t2e[j] = (int32_t)(std::lower_bound(uk.begin(), uk.end(), ek[j]) - uk.begin());
  std::vector<uint64_t>().swap(ek);
  std::vector<uint64_t>().swap(uk);
  // ---- faces
  std::vector<FaceKey> fk(4 * (size_t)nt);
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < nt; ++t)
    for (int lf = 0; lf < 4; ++lf) {
      const int32_t* v = &T.ts[4 * (size_t)t];
      fk[4 * (size_t)t + lf] = {(uint64_t)v[LF[lf][0]] * unv + (uint64_t)v[LF[lf][1]],
                                (uint32_t)v[LF[lf][2]], (uint32_t)(4 * t + lf)};
    }
  std::sort(fk.begin(), fk.end(), [](const FaceKey& a, const FaceKey& b) {
    if (a.ab != b.ab) return a.ab < b.ab;
    if (a.c != b.c) return a.c < b.c;
    return a.occ < b.occ;
  });
  T.nbr.assign(4 * (size_t)nt, -1);
  T.bf_of.assign(4 * (size_t)nt, -1);
  T.nfaces = 0;
  for (size_t i = 0; i < fk.size();) {
    size_t j = i + 1;
    while (j < fk.size() && fk[j].ab == fk[i].ab && fk[j].c == fk[i].c) ++j;
    if (j - i == 1) {
      T.bf_of[fk[i].occ] = (int32_t)T.bf_tet.size();
      T.bf_tet.push_back((int32_t)(fk[i].occ / 4));
      T.bf_lf.push_back((int32_t)(fk[i].occ % 4));
    } else if (j - i == 2) {
      T.nbr[fk[i].occ] = (int32_t)(fk[i + 1].occ / 4);
      T.nbr[fk[i + 1].occ] = (int32_t)(fk[i].occ / 4);
    } else {
      return "non-manifold face shared by more than two tetrahedra";
    }
    T.nfaces++;
    i = j;
  }
  T.nbf = (int64_t)T.bf_tet.size();
  std::vector<FaceKey>().swap(fk);
  // ---- incidences
  bucket(T.ne, T.t2e, 6, T.e2t_ptr, T.e2t);
  bucket(nv, T.ts, 4, T.v2t_ptr, T.v2t);
  // ---- CSR pattern: edges sharing a tetrahedron
  T.row_ptr.assign(T.ne + 1, 0);
  std::vector<std::vector<int32_t>> rows_tmp;
#pragma omp parallel
  {
    std::vector<int32_t> cand;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t e = 0; e < T.ne; ++e) {
      cand.clear();
      for (int64_t k = T.e2t_ptr[e]; k < T.e2t_ptr[e + 1]; ++k)
        for (int q = 0; q < 6; ++q) cand.push_back(T.t2e[6 * (size_t)T.e2t[k] + q]);
      std::sort(cand.begin(), cand.end());
      T.row_ptr[e + 1] = (int64_t)(std::unique(cand.begin(), cand.end()) - cand.begin());
    }
  }
  for (int64_t e = 0; e < T.ne; ++e) T.row_ptr[e + 1] += T.row_ptr[e];
  T.nnz = T.row_ptr[T.ne];
  T.col.resize(T.nnz);
#pragma omp parallel
  {
    std::vector<int32_t> cand;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t e = 0; e < T.ne; ++e) {
      cand.clear();
      for (int64_t k = T.e2t_ptr[e]; k < T.e2t_ptr[e + 1]; ++k)
        for (int q = 0; q < 6; ++q) cand.push_back(T.t2e[6 * (size_t)T.e2t[k] + q]);
      std::sort(cand.begin(), cand.end());
      auto end = std::unique(cand.begin(), cand.end());
      std::copy(cand.begin(), end, T.col.begin() + T.row_ptr[e]);
    }
  }
  // ---- contributions: tetrahedra ascending, then boundary faces ascending
  auto pos_of = [&](int64_t r, int32_t c) -> int64_t {
    auto b = T.col.begin() + T.row_ptr[r], en = T.col.begin() + T.row_ptr[r + 1];
    return (int64_t)(std::lower_bound(b, en, c) - T.col.begin());
  };
  std::vector<int32_t> cnt(T.nnz, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t e = 0; e < T.ne; ++e)
    for (int64_t k = T.e2t_ptr[e]; k < T.e2t_ptr[e + 1]; ++k) {
      const int32_t* te = &T.t2e[6 * (size_t)T.e2t[k]];
      for (int q = 0; q < 6; ++q) cnt[pos_of(e, te[q])]++;
    }
  for (int64_t f = 0; f < T.nbf; ++f) {
    const int32_t* te = &T.t2e[6 * (size_t)T.bf_tet[f]];
    const int* fe = FE[T.bf_lf[f]];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) cnt[pos_of(te[fe[p]], te[fe[q]])]++;
  }
  T.cptr.assign(T.nnz + 1, 0);
  for (int64_t i = 0; i < T.nnz; ++i) T.cptr[i + 1] = T.cptr[i] + cnt[i];
  T.csrc.resize(T.cptr[T.nnz]);
  std::vector<int64_t> cur(T.cptr.begin(), T.cptr.end() - 1);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t e = 0; e < T.ne; ++e)
    for (int64_t k = T.e2t_ptr[e]; k < T.e2t_ptr[e + 1]; ++k) {
      int32_t t = T.e2t[k];
      const int32_t* te = &T.t2e[6 * (size_t)t];
      int p = 0;
      while (te[p] != e) ++p;
      for (int q = 0; q < 6; ++q) T.csrc[cur[pos_of(e, te[q])]++] = 36 * t + 6 * p + q;
    }
  const int64_t fbase = 36 * (int64_t)nt;
  if (fbase + 9 * T.nbf >= (int64_t)INT32_MAX) return "mesh too large for 32-bit source indices";
  for (int64_t f = 0; f < T.nbf; ++f) {
    const int32_t* te = &T.t2e[6 * (size_t)T.bf_tet[f]];
    const int* fe = FE[T.bf_lf[f]];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        T.csrc[cur[pos_of(te[fe[p]], te[fe[q]])]++] = (int32_t)(fbase + 9 * f + 3 * p + q);
  }
  return "";
}

// --------------------------------------------------------------------------

namespace {

void rcb_split(const std::vector<double>& cen, std::vector<int32_t>& ids, size_t lo, size_t hi,
               int32_t p0, int32_t np, std::vector<int32_t>& part) {
  if (np == 1) {
    for (size_t k = lo; k < hi; ++k) part[ids[k]] = p0;
    return;
  }
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx_[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (size_t k = lo; k < hi; ++k)
    for (int c = 0; c < 3; ++c) {
      double v = cen[3 * (size_t)ids[k] + c];
      mn[c] = std::min(mn[c], v);
      mx_[c] = std::max(mx_[c], v);
    }
  int ax = 0;
  double best = mx_[0] - mn[0];
  for (int c = 1; c < 3; ++c)
    if (mx_[c] - mn[c] > best) { best = mx_[c] - mn[c]; ax = c; }
  std::sort(ids.begin() + lo, ids.begin() + hi, [&](int32_t a, int32_t b) {
    double ca = cen[3 * (size_t)a + ax], cb = cen[3 * (size_t)b + ax];
    if (ca != cb) return ca < cb;
    return a < b;
  });
  size_t mid = lo + (hi - lo) / 2;
  rcb_split(cen, ids, lo, mid, p0, np / 2, part);
  rcb_split(cen, ids, mid, hi, p0 + np / 2, np / 2, part);
}

}  // namespace

// Reverse Cuthill-McKee order of a graph given as CSR (ptr, adj) on n nodes
// (Cuthill & McKee 1969, reversed as proposed by George 1971): breadth-first
// from a pseudo-peripheral start node (the end of repeated breadth-first
// sweeps from a node of minimum degree), neighbours visited by increasing
// degree then index; every connected component in turn. Returns order[k] =
// node placed at position k.
static std::vector<int32_t> rcm_order(int32_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj) {
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> level(n, -1);
  std::vector<char> placed(n, 0);
  auto deg = [&](int32_t v) { return (int32_t)(ptr[v + 1] - ptr[v]); };
  // breadth-first levels from r over the unplaced nodes; returns the last node
  // of the deepest level with minimum degree, and the depth
  std::vector<int32_t> q, comp;
  auto bfs = [&](int32_t r, int32_t& depth) {
    for (int32_t v : comp) level[v] = -1;
    comp.clear();
    q.clear();
    q.push_back(r);
    level[r] = 0;
    comp.push_back(r);
    for (size_t h = 0; h < q.size(); ++h) {
      const int32_t v = q[h];
      for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
        const int32_t u = adj[e];
        if (placed[u] || level[u] >= 0) continue;
        level[u] = level[v] + 1;
        q.push_back(u);
        comp.push_back(u);
      }
    }
    depth = level[q.back()];
    int32_t best = q.back();
    for (int32_t v : q)
      if (level[v] == depth && (deg(v) < deg(best) || (deg(v) == deg(best) && v < best))) best = v;
    return best;
  };
  for (int32_t seed = 0; seed < n; ++seed) {
    if (placed[seed]) continue;
    // node of minimum degree in seed's component, then pseudo-peripheral
    int32_t depth = 0;
    bfs(seed, depth);
    int32_t r = seed;
    for (int32_t v : comp)
      if (deg(v) < deg(r) || (deg(v) == deg(r) && v < r)) r = v;
    int32_t d0 = -1;
    for (int it = 0; it < 8; ++it) {
      int32_t d = 0;
      const int32_t far = bfs(r, d);
      if (d <= d0) break;
      d0 = d;
      r = far;
    }
    for (int32_t v : comp) level[v] = -1;
    comp.clear();
    // Cuthill-McKee from r
    const size_t start = order.size();
    order.push_back(r);
    placed[r] = 1;
    std::vector<int32_t> nb;
    for (size_t h = start; h < order.size(); ++h) {
      const int32_t v = order[h];
      nb.clear();
      for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
        if (!placed[adj[e]]) nb.push_back(adj[e]);
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg(a) < deg(b) || (deg(a) == deg(b) && a < b); });
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      for (int32_t u : nb) {
        placed[u] = 1;
        order.push_back(u);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

std::string build_decomposition(const Topology& T, int32_t nsub, int32_t overlap, int32_t nb,
                                Decomposition& Dc) {
  if (nsub < 1 || (nsub & (nsub - 1))) return "nsub must be a power of two";
  if (overlap < 1) return "overlap must be >= 1";
  if (nsub > T.nt) return "more subdomains than tetrahedra";
  Dc = Decomposition();
  Dc.nsub = nsub;
  Dc.overlap = overlap;
  Dc.nb = nb;
  const int32_t nt = T.nt, nv = T.nv;
  // centroids in input vertex order
  std::vector<double> cen(3 * (size_t)nt);
  for (int32_t t = 0; t < nt; ++t)
    for (int c = 0; c < 3; ++c) {
      const int32_t* v = &T.tet_in[4 * (size_t)t];
      cen[3 * (size_t)t + c] = (((T.xyz[3 * (size_t)v[0] + c] + T.xyz[3 * (size_t)v[1] + c]) +
                                 T.xyz[3 * (size_t)v[2] + c]) +
                                T.xyz[3 * (size_t)v[3] + c]) *
                               0.25;
    }
  Dc.part.assign(nt, 0);
  std::vector<int32_t> ids(nt);
  std::iota(ids.begin(), ids.end(), 0);
  rcb_split(cen, ids, 0, nt, 0, nsub, Dc.part);
  std::vector<int64_t> pptr;
  std::vector<int32_t> ptets;
  bucket(nsub, Dc.part, 1, pptr, ptets);

  std::vector<std::vector<int32_t>> sub_tets(nsub), sub_dofs(nsub), sub_w(nsub);
#pragma omp parallel
  {
    std::vector<int32_t> layer(nv, -1);
    std::vector<char> inT(nt, 0), inE(T.ne, 0);
    std::vector<int32_t> vtouched, frontier, next, tl;
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < nsub; ++i) {
      tl.assign(ptets.begin() + pptr[i], ptets.begin() + pptr[i + 1]);
      vtouched.clear();
      frontier.clear();
      for (int32_t t : tl) {
        inT[t] = 1;
        for (int k = 0; k < 4; ++k) {
          int32_t v = T.ts[4 * (size_t)t + k];
          if (layer[v] < 0) { layer[v] = 0; vtouched.push_back(v); frontier.push_back(v); }
        }
      }
      for (int l = 1; l <= overlap; ++l) {
        std::vector<int32_t> newt;
        for (int32_t v : frontier)
          for (int64_t k = T.v2t_ptr[v]; k < T.v2t_ptr[v + 1]; ++k) {
            int32_t t = T.v2t[k];
            if (!inT[t]) { inT[t] = 1; newt.push_back(t); }
          }
        next.clear();
        for (int32_t t : newt) {
          tl.push_back(t);
          for (int k = 0; k < 4; ++k) {
            int32_t v = T.ts[4 * (size_t)t + k];
            if (layer[v] < 0) { layer[v] = l; vtouched.push_back(v); next.push_back(v); }
          }
        }
        frontier.swap(next);
      }
      std::sort(tl.begin(), tl.end());
      std::vector<int32_t> dl;
      for (int32_t t : tl)
        for (int q = 0; q < 6; ++q) {
          int32_t e = T.t2e[6 * (size_t)t + q];
          if (!inE[e]) { inE[e] = 1; dl.push_back(e); }
        }
      std::sort(dl.begin(), dl.end());
      std::vector<int32_t> wl(dl.size());
      for (size_t k = 0; k < dl.size(); ++k) {
        int32_t a = T.edges[2 * (size_t)dl[k]], b = T.edges[2 * (size_t)dl[k] + 1];
        int32_t wa = std::max(overlap - layer[a], 0), wb = std::max(overlap - layer[b], 0);
        wl[k] = wa + wb;
      }
      for (int32_t e : dl) inE[e] = 0;
      for (int32_t t : tl) inT[t] = 0;
      for (int32_t v : vtouched) layer[v] = -1;
      sub_tets[i].swap(tl);
      sub_dofs[i].swap(dl);
      sub_w[i].swap(wl);
      tl.clear();
    }
  }
  Dc.dof_ptr.assign(nsub + 1, 0);
  Dc.tet_ptr.assign(nsub + 1, 0);
  for (int32_t i = 0; i < nsub; ++i) {
    Dc.dof_ptr[i + 1] = Dc.dof_ptr[i] + (int64_t)sub_dofs[i].size();
    Dc.tet_ptr[i + 1] = Dc.tet_ptr[i] + (int64_t)sub_tets[i].size();
  }
  Dc.dofs.resize(Dc.dof_ptr[nsub]);
  Dc.w.resize(Dc.dof_ptr[nsub]);
  Dc.tets.resize(Dc.tet_ptr[nsub]);
  for (int32_t i = 0; i < nsub; ++i) {
    std::copy(sub_dofs[i].begin(), sub_dofs[i].end(), Dc.dofs.begin() + Dc.dof_ptr[i]);
    std::copy(sub_w[i].begin(), sub_w[i].end(), Dc.w.begin() + Dc.dof_ptr[i]);
    std::copy(sub_tets[i].begin(), sub_tets[i].end(), Dc.tets.begin() + Dc.tet_ptr[i]);
  }
  std::vector<int64_t> wsum(T.ne, 0);
  for (int64_t k = 0; k < Dc.dof_ptr[nsub]; ++k) wsum[Dc.dofs[k]] += Dc.w[k];
  for (int64_t e = 0; e < T.ne; ++e)
    if (wsum[e] <= 0) return "partition of unity leaves an edge uncovered";
  Dc.D.resize(Dc.dof_ptr[nsub]);
  for (int64_t k = 0; k < Dc.dof_ptr[nsub]; ++k)
    Dc.D[k] = (double)Dc.w[k] / (double)wsum[Dc.dofs[k]];
  // ---- adjacency (shared DOFs) and greedy colouring
  std::vector<int32_t> owner_sub(Dc.dof_ptr[nsub]);
  for (int32_t i = 0; i < nsub; ++i)
    for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) owner_sub[k] = i;
  std::vector<int64_t> es_ptr(T.ne + 1, 0);
  for (int64_t k = 0; k < Dc.dof_ptr[nsub]; ++k) es_ptr[Dc.dofs[k] + 1]++;
  for (int64_t e = 0; e < T.ne; ++e) es_ptr[e + 1] += es_ptr[e];
  std::vector<int32_t> es(Dc.dof_ptr[nsub]);
  {
    std::vector<int64_t> c(es_ptr.begin(), es_ptr.end() - 1);
    for (int64_t k = 0; k < Dc.dof_ptr[nsub]; ++k) es[c[Dc.dofs[k]]++] = owner_sub[k];
  }
  std::vector<std::vector<int32_t>> adj(nsub);
  for (int64_t e = 0; e < T.ne; ++e)
    for (int64_t a = es_ptr[e]; a < es_ptr[e + 1]; ++a)
      for (int64_t b = es_ptr[e]; b < es_ptr[e + 1]; ++b)
        if (a != b) adj[es[a]].push_back(es[b]);
  Dc.nbr_ptr.assign(nsub + 1, 0);
  for (int32_t i = 0; i < nsub; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    Dc.nbr_ptr[i + 1] = Dc.nbr_ptr[i] + (int64_t)adj[i].size();
  }
  for (int32_t i = 0; i < nsub; ++i) Dc.nbrs.insert(Dc.nbrs.end(), adj[i].begin(), adj[i].end());
  Dc.colour.assign(nsub, -1);
  Dc.ncolour = 0;
  for (int32_t i = 0; i < nsub; ++i) {
    std::vector<char> used(nsub + 1, 0);
    for (int32_t j : adj[i])
      if (Dc.colour[j] >= 0) used[Dc.colour[j]] = 1;
    int32_t c = 0;
    while (used[c]) ++c;
    Dc.colour[i] = c;
    Dc.ncolour = std::max(Dc.ncolour, c + 1);
  }
  // ---- padded dense sizes
  Dc.Npad.resize(nsub);
  Dc.mat_off.assign(nsub + 1, 0);
  Dc.vec_off.assign(nsub + 1, 0);
  for (int32_t i = 0; i < nsub; ++i) {
    int64_t n = Dc.dof_ptr[i + 1] - Dc.dof_ptr[i];
    int64_t N = (n + nb - 1) / nb * nb;
    Dc.Npad[i] = (int32_t)N;
    Dc.mat_off[i + 1] = Dc.mat_off[i] + N * N;
    Dc.vec_off[i + 1] = Dc.vec_off[i] + N;
  }
  // ---- dense order of each subdomain's DOFs: reverse Cuthill-McKee on the
  // graph of DOFs that share a tetrahedron of the subdomain
  Dc.lpos.assign(Dc.dof_ptr[nsub], 0);
  Dc.dense_edge.assign(Dc.vec_off[nsub], -1);
  Dc.band_np = 0;
  for (int32_t i = 0; i < nsub; ++i) Dc.band_np = std::max(Dc.band_np, Dc.Npad[i] / nb);
  Dc.band0.assign((size_t)nsub * Dc.band_np, -1);
#pragma omp parallel
  {
    std::vector<int32_t> loc(T.ne, -1);
    std::vector<std::pair<int32_t, int32_t>> pairs;
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < nsub; ++i) {
      const int32_t n = (int32_t)(Dc.dof_ptr[i + 1] - Dc.dof_ptr[i]);
      for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) loc[Dc.dofs[k]] = (int32_t)(k - Dc.dof_ptr[i]);
      pairs.clear();
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) {
        const int32_t* te = &T.t2e[6 * (size_t)Dc.tets[k]];
        for (int a = 0; a < 6; ++a)
          for (int b = 0; b < 6; ++b)
            if (a != b) pairs.push_back({loc[te[a]], loc[te[b]]});
      }
      std::sort(pairs.begin(), pairs.end());
      pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
      std::vector<int64_t> ptr(n + 1, 0);
      std::vector<int32_t> adj(pairs.size());
      for (auto& pr : pairs) ptr[pr.first + 1]++;
      for (int32_t v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
      for (size_t e = 0; e < pairs.size(); ++e) adj[e] = pairs[e].second;
      const std::vector<int32_t> ord = rcm_order(n, ptr, adj);
      for (int32_t r = 0; r < n; ++r) {
        Dc.lpos[Dc.dof_ptr[i] + ord[r]] = r;
        Dc.dense_edge[Dc.vec_off[i] + r] = Dc.dofs[Dc.dof_ptr[i] + ord[r]];
      }
      // structural band: last row of each dense column (the diagonal, the
      // padding identity and every pair of DOFs sharing a tetrahedron)
      const int32_t Ni = Dc.Npad[i];
      std::vector<int32_t> colmax(Ni);
      for (int32_t r = 0; r < Ni; ++r) colmax[r] = r;
      for (auto& pr : pairs) {
        const int32_t ra = Dc.lpos[Dc.dof_ptr[i] + pr.first], rb = Dc.lpos[Dc.dof_ptr[i] + pr.second];
        colmax[rb] = std::max(colmax[rb], ra);
      }
      for (int32_t c = 0; c < Ni; ++c) {
        int32_t& b = Dc.band0[(size_t)i * Dc.band_np + c / nb];
        b = std::max(b, colmax[c] / nb);
      }
      for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) loc[Dc.dofs[k]] = -1;
    }
  }
  // ---- interface faces
  {
    std::vector<int64_t> keys;
    std::vector<char> inT(nt, 0);
    for (int32_t i = 0; i < nsub; ++i) {
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) inT[Dc.tets[k]] = 1;
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) {
        int32_t t = Dc.tets[k];
        for (int lf = 0; lf < 4; ++lf) {
          int32_t o = T.nbr[4 * (size_t)t + lf];
          if (o >= 0 && !inT[o]) keys.push_back(4 * (int64_t)t + lf);
        }
      }
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) inT[Dc.tets[k]] = 0;
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (int64_t k : keys) {
      Dc.if_tet.push_back((int32_t)(k / 4));
      Dc.if_lf.push_back((int32_t)(k % 4));
    }
  }
  const int64_t fbase = 36 * (int64_t)nt;
  const int64_t ibase = fbase + 9 * T.nbf;
  if (ibase + 9 * (int64_t)Dc.if_tet.size() >= (int64_t)INT32_MAX)
    return "mesh too large for 32-bit source indices";
  // ---- local assembly lists
  std::vector<std::vector<int64_t>> sdest(nsub), sptr(nsub);
  std::vector<std::vector<int32_t>> ssrc(nsub);
#pragma omp parallel
  {
    std::vector<int32_t> loc(T.ne, -1);
    std::vector<char> inT(nt, 0);
    std::vector<std::pair<int64_t, int32_t>> items;
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < nsub; ++i) {
      const int64_t N = Dc.Npad[i];
      for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) loc[Dc.dofs[k]] = Dc.lpos[k];  // dense row
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) inT[Dc.tets[k]] = 1;
      items.clear();
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) {
        int32_t t = Dc.tets[k];
        const int32_t* te = &T.t2e[6 * (size_t)t];
        for (int p = 0; p < 6; ++p)
          for (int q = 0; q < 6; ++q)
            items.push_back({(int64_t)loc[te[p]] * N + loc[te[q]], 36 * t + 6 * p + q});
      }
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) {
        int32_t t = Dc.tets[k];
        const int32_t* te = &T.t2e[6 * (size_t)t];
        for (int lf = 0; lf < 4; ++lf) {
          int32_t o = T.nbr[4 * (size_t)t + lf];
          int64_t base;
          if (o < 0) {
            base = fbase + 9 * (int64_t)T.bf_of[4 * (size_t)t + lf];
          } else if (!inT[o]) {
            int64_t key = 4 * (int64_t)t + lf;
            // binary search in the interface list (sorted by tet, face)
            int64_t lo = 0, hi = (int64_t)Dc.if_tet.size();
            while (lo < hi) {
              int64_t m = (lo + hi) / 2;
              int64_t km = 4 * (int64_t)Dc.if_tet[m] + Dc.if_lf[m];
              if (km < key) lo = m + 1; else hi = m;
            }
            base = ibase + 9 * lo;
          } else {
            continue;
          }
          const int* fe = FE[lf];
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
              items.push_back({(int64_t)loc[te[fe[p]]] * N + loc[te[fe[q]]],
                               (int32_t)(base + 3 * p + q)});
        }
      }
      std::stable_sort(items.begin(), items.end(),
                       [](const std::pair<int64_t, int32_t>& a, const std::pair<int64_t, int32_t>& b) {
                         return a.first < b.first;
                       });
      std::vector<int64_t> d, pp;
      std::vector<int32_t> s;
      s.reserve(items.size());
      for (size_t a = 0; a < items.size();) {
        size_t b = a;
        d.push_back(Dc.mat_off[i] + items[a].first);
        pp.push_back((int64_t)s.size());
        while (b < items.size() && items[b].first == items[a].first) s.push_back(items[b++].second);
        a = b;
      }
      sdest[i].swap(d);
      sptr[i].swap(pp);
      ssrc[i].swap(s);
      for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) loc[Dc.dofs[k]] = -1;
      for (int64_t k = Dc.tet_ptr[i]; k < Dc.tet_ptr[i + 1]; ++k) inT[Dc.tets[k]] = 0;
    }
  }
  int64_t nloc = 0, ncon = 0;
  for (int32_t i = 0; i < nsub; ++i) {
    nloc += (int64_t)sdest[i].size();
    ncon += (int64_t)ssrc[i].size();
  }
  Dc.ldest.reserve(nloc);
  Dc.lptr.reserve(nloc + 1);
  Dc.lsrc.reserve(ncon);
  for (int32_t i = 0; i < nsub; ++i) {
    int64_t base = (int64_t)Dc.lsrc.size();
    Dc.ldest.insert(Dc.ldest.end(), sdest[i].begin(), sdest[i].end());
    for (int64_t v : sptr[i]) Dc.lptr.push_back(base + v);
    Dc.lsrc.insert(Dc.lsrc.end(), ssrc[i].begin(), ssrc[i].end());
  }
  Dc.lptr.push_back((int64_t)Dc.lsrc.size());
  // ---- prolongation lists by colour
  Dc.pcol_ptr.assign(Dc.ncolour + 1, 0);
  for (int32_t c = 0; c < Dc.ncolour; ++c) {
    for (int32_t i = 0; i < nsub; ++i) {
      if (Dc.colour[i] != c) continue;
      for (int64_t k = Dc.dof_ptr[i]; k < Dc.dof_ptr[i + 1]; ++k) {
        if (Dc.w[k] == 0) continue;
        Dc.p_edge.push_back(Dc.dofs[k]);
        Dc.p_row.push_back(Dc.vec_off[i] + Dc.lpos[k]);
        Dc.p_w.push_back(Dc.D[k]);
      }
    }
    Dc.pcol_ptr[c + 1] = (int64_t)Dc.p_edge.size();
  }
  // ---- the same entries by destination edge (stable: colour order kept)
  const size_t np = Dc.p_edge.size();
  Dc.pg_ptr.assign(T.ne + 1, 0);
  for (size_t k = 0; k < np; ++k) ++Dc.pg_ptr[Dc.p_edge[k] + 1];
  for (int64_t e = 0; e < T.ne; ++e) Dc.pg_ptr[e + 1] += Dc.pg_ptr[e];
  Dc.pg_row.resize(np);
  Dc.pg_w.resize(np);
  std::vector<int64_t> fill(Dc.pg_ptr.begin(), Dc.pg_ptr.end() - 1);
  for (size_t k = 0; k < np; ++k) {
    const int64_t q = fill[Dc.p_edge[k]]++;
    Dc.pg_row[q] = Dc.p_row[k];
    Dc.pg_w[q] = Dc.p_w[k];
  }
  return "";
}

// --------------------------------------------------------------------------

bool point_functional(const Topology& T, const double x[3], const double p_re[3],
                      const double p_im[3], std::vector<int32_t>& edge,
                      std::vector<double>& val) {
  std::vector<int32_t> hits;
#pragma omp parallel
  {
    std::vector<int32_t> mine;
#pragma omp for schedule(static) nowait
    for (int32_t t = 0; t < T.nt; ++t) {
      const int32_t* v = &T.ts[4 * (size_t)t];
      bool in = true;
      for (int k = 0; k < 4 && in; ++k) {
        // barycentric k from the normal of the opposite face
        int j[3], m = 0;
        for (int q = 0; q < 4; ++q)
          if (q != k) j[m++] = q;
        const double* a = &T.xyz[3 * (size_t)v[j[0]]];
        const double* b = &T.xyz[3 * (size_t)v[j[1]]];
        const double* c = &T.xyz[3 * (size_t)v[j[2]]];
        const double* pk = &T.xyz[3 * (size_t)v[k]];
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        double den = n[0] * (pk[0] - a[0]) + n[1] * (pk[1] - a[1]) + n[2] * (pk[2] - a[2]);
        double num = n[0] * (x[0] - a[0]) + n[1] * (x[1] - a[1]) + n[2] * (x[2] - a[2]);
        if (num / den < -1e-12) in = false;
      }
      if (in) mine.push_back(t);
    }
#pragma omp critical
    hits.insert(hits.end(), mine.begin(), mine.end());
  }
  std::sort(hits.begin(), hits.end());
  edge.clear();
  val.clear();
  if (hits.empty()) return false;
  std::vector<std::pair<int32_t, std::pair<double, double>>> acc;
  for (int32_t t : hits) {
    const int32_t* v = &T.ts[4 * (size_t)t];
    double lam[4], g[4][3];
    for (int k = 0; k < 4; ++k) {
      int j[3], m = 0;
      for (int q = 0; q < 4; ++q)
        if (q != k) j[m++] = q;
      const double* a = &T.xyz[3 * (size_t)v[j[0]]];
      const double* b = &T.xyz[3 * (size_t)v[j[1]]];
      const double* c = &T.xyz[3 * (size_t)v[j[2]]];
      const double* pk = &T.xyz[3 * (size_t)v[k]];
      double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      double den = n[0] * (pk[0] - a[0]) + n[1] * (pk[1] - a[1]) + n[2] * (pk[2] - a[2]);
      for (int d = 0; d < 3; ++d) g[k][d] = n[d] / den;
      lam[k] = (n[0] * (x[0] - a[0]) + n[1] * (x[1] - a[1]) + n[2] * (x[2] - a[2])) / den;
    }
    for (int le = 0; le < 6; ++le) {
      int a = LE[le][0], b = LE[le][1];
      double re = 0, im = 0;
      for (int d = 0; d < 3; ++d) {
        double N = lam[a] * g[b][d] - lam[b] * g[a][d];
        re += p_re[d] * N;
        im += p_im[d] * N;
      }
      acc.push_back({T.t2e[6 * (size_t)t + le], {re, im}});
    }
  }
  std::stable_sort(acc.begin(), acc.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  const double inv = 1.0 / (double)hits.size();
  for (size_t a = 0; a < acc.size();) {
    size_t b = a;
    double re = 0, im = 0;
    while (b < acc.size() && acc[b].first == acc[a].first) {
      re += acc[b].second.first;
      im += acc[b].second.second;
      ++b;
    }
    edge.push_back(acc[a].first);
    val.push_back(re * inv);
    val.push_back(im * inv);
    a = b;
  }
  return true;
}

bool build_col_windows(const Topology& T, int32_t cap, int32_t max_rows, ColWindows& W) {
  W = ColWindows();
  const int64_t n = T.ne;
  if (n <= 0 || cap <= 0 || cap > 256 || max_rows <= 0) return false;
  for (int64_t r = 0; r < n; ++r)
    if (T.row_ptr[r + 1] - T.row_ptr[r] > cap) return false;
  std::vector<int32_t> mark(n, -1);   // slice that last counted the column
  std::vector<int32_t> cols;
  W.cap = cap;
  W.max_rows = max_rows;
  W.row.push_back(0);
  W.cptr.push_back(0);
  W.lcol.resize(T.nnz);
  int64_t r = 0;
  for (int32_t s = 0; r < n; ++s) {
    const int64_t r0 = r;
    int32_t u = 0;
    while (r < n && r - r0 < max_rows) {
      int32_t fresh = 0;
      for (int64_t k = T.row_ptr[r]; k < T.row_ptr[r + 1]; ++k) fresh += mark[T.col[k]] != s;
      if (u + fresh > cap) break;
      for (int64_t k = T.row_ptr[r]; k < T.row_ptr[r + 1]; ++k)
        if (mark[T.col[k]] != s) {
          mark[T.col[k]] = s;
          ++u;
        }
      ++r;
    }
    cols.assign(T.col.begin() + T.row_ptr[r0], T.col.begin() + T.row_ptr[r]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int64_t k = T.row_ptr[r0]; k < T.row_ptr[r]; ++k)
      W.lcol[k] = (uint8_t)(std::lower_bound(cols.begin(), cols.end(), T.col[k]) - cols.begin());
    W.ucol.insert(W.ucol.end(), cols.begin(), cols.end());
    W.umax = std::max(W.umax, (int32_t)cols.size());
    W.row.push_back((int32_t)r);
    W.cptr.push_back((int32_t)W.ucol.size());
  }
  return true;
}

}  // namespace mx
