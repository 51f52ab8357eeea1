// Host construction of the periodic tree and its interaction lists.
//
// Tree (Sec. 3.1): every fibre owns a basic tree whose root is the lattice
// cell, a square of side a centred on the fibre; a cell holding more than
// leaf_max element midpoints is cut into quadrants (half-open intervals).
// Cells keep their geometric centre (so translation vectors repeat across
// the lattice) and a tight radius rho that bounds every chord in the cell.
//
// Lists: for a target fibre i, a source fibre j and an image m (source
// shifted by m h), the pair of roots is "far" (Sec. 3.1, far basic trees)
// when 2 rho_max <= mac |c_i - c_j - m h|; all far images of (i, j) are
// folded into one top-level M2L with the lattice sum S(c_i - c_j)
// (Sec. 3.3).  The remaining (adjacent) images are finitely many; for each
// of them a dual traversal of the two trees emits M2L pairs where
// rho_D + rho_C <= mac |O_D - O_C - m h| and P2P pairs between leaves that
// are not separated.  Pairs with j = i and m = 0 also form the lists of the
// interior (wavenumber k1) operators, which act within one fibre only; they
// are left out when that block is applied by FFT (Problem::self_fft).
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <memory>
#include <utility>

#include "pfm_internal.hpp"

namespace pfm {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on the Legendre polynomial P_n from Chebyshev-like guesses.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // final derivative at the converged node
        double q0 = 1.0, q1 = z;
        for (int k = 2; k <= n; ++k) {
          double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
          q0 = q1;
          q1 = q2;
        }
        if (n == 1) { q1 = z; q0 = 1.0; }
        dp = n * (z * q1 - q0) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
    }
  }
}

namespace {

struct TCell {
  double cx, cy, half, rho = 0.0;
  int shape = 0;               // 0 square, 1 hexagon (triangle-tree root), 2 triangle
  double vx[3] = {0, 0, 0}, vy[3] = {0, 0, 0};   // a triangle's corners
  int level, fiber;
  int parent = -1;
  std::vector<int> kids;       // tmp ids
  std::vector<int> elems;      // natural element ids
  int id = -1;                 // final id
};

struct KeyHash {
  std::map<std::pair<long long, long long>, int> m;
  std::vector<double>* xy;
  int get(double dx, double dy, double scale) {
    auto key = std::make_pair(std::llround(dx * scale), std::llround(dy * scale));
    auto it = m.find(key);
    if (it != m.end()) return it->second;
    int id = (int)(xy->size() / 2);
    xy->push_back(dx);
    xy->push_back(dy);
    m.emplace(key, id);
    return id;
  }
};

}  // namespace

bool build_host_plan(Problem& pb, const std::vector<double>& mid, const std::vector<double>& ends) {
  HostPlan& hp = pb.hp;
  const int M = pb.M, N = pb.N;
  const int leaf_max = pb.opt.leaf_max;
  const double mac = pb.opt.mac;
  std::vector<TCell> tc;
  tc.reserve(M * 64);
  std::vector<int> roots(M);

  std::function<void(int)> split;
  // Triangle quadtree of the hexagonal lattice (Sec. 3.1, Fig. 5): the
  // root is the fibre's hexagonal lattice cell, cut into six equilateral
  // triangles (centre and two neighbouring corners); a triangle is cut into
  // four by its edge midpoints (three corner triangles and the inverted
  // middle one).  An element goes where its midpoint lies: the sextant of its
  // angle about the centre, then by barycentric coordinates (corner i when
  // l_i >= 1/2, else the middle).  A cell's centre is its centroid (the
  // hexagon's is the fibre centre).
  auto add_tri = [&](int parent, const double* x, const double* y) {
    TCell c;
    c.shape = 2;
    for (int v = 0; v < 3; ++v) {
      c.vx[v] = x[v];
      c.vy[v] = y[v];
    }
    c.cx = (x[0] + x[1] + x[2]) / 3.0;
    c.cy = (y[0] + y[1] + y[2]) / 3.0;
    c.half = 0.5 * std::hypot(x[1] - x[0], y[1] - y[0]);
    c.level = tc[parent].level + 1;
    c.fiber = tc[parent].fiber;
    c.parent = parent;
    tc.push_back(c);
    return (int)tc.size() - 1;
  };
  std::function<void(int)> split_triangles = [&](int id) {
    std::vector<int> kid(6, -1), elems = tc[id].elems;
    const TCell p = tc[id];
    for (int e : elems) {
      const double px = mid[2 * e], py = mid[2 * e + 1];
      int q;
      double x[3], y[3];
      if (p.shape == 1) {
        // sextant s between the corners at angles 60 s and 60 (s + 1) degrees
        double ang = std::atan2(py - p.cy, px - p.cx);
        if (ang < 0) ang += 2.0 * PI;
        q = std::min(5, (int)std::floor(ang / (PI / 3.0)));
        const double R = p.half;            // circumradius of the hexagon
        x[0] = p.cx; y[0] = p.cy;
        x[1] = p.cx + R * std::cos(q * PI / 3.0); y[1] = p.cy + R * std::sin(q * PI / 3.0);
        x[2] = p.cx + R * std::cos((q + 1) * PI / 3.0); y[2] = p.cy + R * std::sin((q + 1) * PI / 3.0);
      } else {
        const double d1x = p.vx[1] - p.vx[0], d1y = p.vy[1] - p.vy[0];
        const double d2x = p.vx[2] - p.vx[0], d2y = p.vy[2] - p.vy[0];
        const double det = d1x * d2y - d1y * d2x;
        const double ex = px - p.vx[0], ey = py - p.vy[0];
        const double l1 = (ex * d2y - ey * d2x) / det, l2 = (d1x * ey - d1y * ex) / det;
        const double l0 = 1.0 - l1 - l2;
        q = l0 >= 0.5 ? 0 : (l1 >= 0.5 ? 1 : (l2 >= 0.5 ? 2 : 3));
        double mx_[3], my_[3];      // midpoints of the edges opposite corner i
        for (int i = 0; i < 3; ++i) {
          mx_[i] = 0.5 * (p.vx[(i + 1) % 3] + p.vx[(i + 2) % 3]);
          my_[i] = 0.5 * (p.vy[(i + 1) % 3] + p.vy[(i + 2) % 3]);
        }
        if (q < 3) {
          // corner q with the midpoints of its two edges, in the parent's orientation
          for (int i = 0; i < 3; ++i) {
            x[i] = i == q ? p.vx[i] : mx_[3 - q - i];
            y[i] = i == q ? p.vy[i] : my_[3 - q - i];
          }
        } else {
          for (int i = 0; i < 3; ++i) {
            x[i] = mx_[i];
            y[i] = my_[i];
          }
        }
      }
      if (kid[q] < 0) kid[q] = add_tri(id, x, y);
      tc[kid[q]].elems.push_back(e);
    }
    for (int q = 0; q < 6; ++q)
      if (kid[q] >= 0) tc[id].kids.push_back(kid[q]);
    std::vector<int> kids = tc[id].kids;
    for (int k : kids) split(k);
  };

  split = [&](int id) {
    // tight radius
    double rho = 0.0;
    for (int e : tc[id].elems) {
      for (int s = 0; s < 2; ++s) {
        double dx = ends[4 * e + 2 * s] - tc[id].cx;
        double dy = ends[4 * e + 2 * s + 1] - tc[id].cy;
        rho = std::max(rho, std::sqrt(dx * dx + dy * dy));
      }
    }
    tc[id].rho = rho;
    if ((int)tc[id].elems.size() <= leaf_max || tc[id].level >= 24) return;
    if (tc[id].shape != 0) {
      split_triangles(id);
      return;
    }
    int kid[4] = {-1, -1, -1, -1};
    std::vector<int> elems = tc[id].elems;
    for (int e : elems) {
      int q = (mid[2 * e] >= tc[id].cx ? 1 : 0) + (mid[2 * e + 1] >= tc[id].cy ? 2 : 0);
      if (kid[q] < 0) {
        TCell c;
        c.half = 0.5 * tc[id].half;
        c.cx = tc[id].cx + ((q & 1) ? c.half : -c.half);
        c.cy = tc[id].cy + ((q & 2) ? c.half : -c.half);
        c.level = tc[id].level + 1;
        c.fiber = tc[id].fiber;
        c.parent = id;
        kid[q] = (int)tc.size();
        tc.push_back(c);
      }
      tc[kid[q]].elems.push_back(e);
    }
    for (int q = 0; q < 4; ++q)
      if (kid[q] >= 0) tc[id].kids.push_back(kid[q]);
    std::vector<int> kids = tc[id].kids;
    for (int k : kids) split(k);
  };

  for (int f = 0; f < M; ++f) {
    TCell r;
    r.cx = pb.centres[2 * f];
    r.cy = pb.centres[2 * f + 1];
    r.half = 0.5 * pb.a;
    if (pb.opt.tree_shape == 1) {
      r.shape = 1;
      r.half = pb.a / std::sqrt(3.0);       // corners of the hexagonal cell (inradius a / 2)
    }
    r.level = 0;
    r.fiber = f;
    for (int e = 0; e < N; ++e) r.elems.push_back(f * N + e);
    roots[f] = (int)tc.size();
    tc.push_back(r);
    split(roots[f]);
  }

  // element order: depth-first per fibre, so every cell owns a contiguous range
  hp.elem_of.clear();
  std::vector<int> ebeg(tc.size()), eend(tc.size());
  std::function<void(int)> dfs = [&](int id) {
    ebeg[id] = (int)hp.elem_of.size();
    if (tc[id].kids.empty()) {
      for (int e : tc[id].elems) hp.elem_of.push_back(e);
    } else {
      for (int k : tc[id].kids) dfs(k);
    }
    eend[id] = (int)hp.elem_of.size();
  };
  for (int f = 0; f < M; ++f) dfs(roots[f]);

  // level-major renumbering; children of one parent stay contiguous
  std::vector<int> order;
  order.insert(order.end(), roots.begin(), roots.end());
  hp.level_beg.assign(1, 0);
  size_t lb = 0;
  int depth = 0;
  while (lb < order.size()) {
    size_t le = order.size();
    hp.level_beg.push_back((int)le);
    for (size_t i = lb; i < le; ++i)
      for (int k : tc[order[i]].kids) order.push_back(k);
    if (order.size() > le) depth++;
    lb = le;
  }
  // level_beg currently has entries at each level end; make it [0, n1, n2, ..., total]
  {
    std::vector<int> beg = {0};
    size_t pos = 0;
    int lvl = 0;
    while (pos < order.size()) {
      size_t e = pos;
      while (e < order.size() && tc[order[e]].level == lvl) e++;
      beg.push_back((int)e);
      pos = e;
      lvl++;
    }
    hp.level_beg = beg;
  }
  hp.depth = (int)hp.level_beg.size() - 2;
  for (size_t i = 0; i < order.size(); ++i) tc[order[i]].id = (int)i;

  const int nc = (int)order.size();
  hp.cells.assign(nc, Cell{});
  hp.leaves.clear();
  for (int i = 0; i < nc; ++i) {
    const TCell& t = tc[order[i]];
    Cell& c = hp.cells[i];
    c.cx = t.cx;
    c.cy = t.cy;
    c.half = t.half;
    c.rho = t.rho;
    c.level = t.level;
    c.fiber = t.fiber;
    c.parent = t.parent >= 0 ? tc[t.parent].id : -1;
    c.n_child = (int)t.kids.size();
    c.first_child = c.n_child ? tc[t.kids[0]].id : -1;
    c.ebeg = ebeg[order[i]];
    c.eend = eend[order[i]];
    c.leaf = c.n_child == 0;
    c.leaf_index = -1;
    if (c.leaf) {
      c.leaf_index = (int)hp.leaves.size();
      hp.leaves.push_back(i);
      // a leaf's rows are the lanes of one wavefront in P2P and L2P;
      // only the level cap can leave more than leaf_max elements in a leaf
      if (c.eend - c.ebeg > 64) return false;
    }
  }
  for (int i = 0; i < nc; ++i) {
    const Cell& c = hp.cells[i];
    for (int k = 0; k < c.n_child; ++k)
      if (c.first_child + k >= nc || hp.cells[c.first_child + k].parent != i) return false;
  }
  hp.root_of_fibre.resize(M);
  for (int f = 0; f < M; ++f) hp.root_of_fibre[f] = tc[roots[f]].id;

  // leaf-to-ancestor offsets: the upward pass gathers, for every non-leaf
  // cell, the leaves below it; the downward pass gathers, for every leaf,
  // its ancestors.  Both use Jp(kap (O_L - O_A)).
  const double scale = std::ldexp(1.0, 36) / pb.a;
  hp.joff_xy.clear();
  KeyHash jh;
  jh.xy = &hp.joff_xy;
  hp.up_cells.clear();
  hp.up_ptr.assign(1, 0);
  hp.up_src.clear();
  hp.up_off.clear();
  {
    std::vector<std::vector<std::pair<int, int>>> below(nc);
    hp.anc_ptr.assign(1, 0);
    hp.anc.clear();
    hp.anc_off.clear();
    for (int l : hp.leaves) {
      const Cell& L = hp.cells[l];
      for (int a = L.parent; a >= 0; a = hp.cells[a].parent) {
        int id = jh.get(L.cx - hp.cells[a].cx, L.cy - hp.cells[a].cy, scale);
        below[a].push_back({l, id});
        hp.anc.push_back(a);
        hp.anc_off.push_back(id);
      }
      hp.anc_ptr.push_back((int)hp.anc.size());
    }
    for (int c = 0; c < nc; ++c) {
      if (hp.cells[c].leaf) continue;
      hp.up_cells.push_back(c);
      for (auto& pr : below[c]) {
        hp.up_src.push_back(pr.first);
        hp.up_off.push_back(pr.second);
      }
      hp.up_ptr.push_back((int)hp.up_src.size());
    }
  }

  // fibre-pair offsets and their explicit image ranges
  double rho_max = 0.0;
  for (int f = 0; f < M; ++f) rho_max = std::max(rho_max, hp.cells[hp.root_of_fibre[f]].rho);
  const double R = 2.0 * rho_max / mac;
  hp.root_off_xy.clear();
  hp.root_off_mrange.clear();
  KeyHash rh;
  rh.xy = &hp.root_off_xy;
  hp.root_pair_off.assign((size_t)M * M, -1);
  for (int i = 0; i < M; ++i) {
    for (int j = 0; j < M; ++j) {
      double ox = pb.centres[2 * i] - pb.centres[2 * j];
      double oy = pb.centres[2 * i + 1] - pb.centres[2 * j + 1];
      size_t before = hp.root_off_xy.size();
      int id = rh.get(ox, oy, scale);
      hp.root_pair_off[(size_t)i * M + j] = id;
      if (hp.root_off_xy.size() != before) {
        // explicit images: 2 rho_max > mac |o - m h|
        int mlo = 1, mhi = 0;
        int mc = (int)std::floor(oy / pb.H);
        int span = (int)std::ceil(R / pb.H) + 2;
        for (int m = mc - span; m <= mc + span; ++m) {
          const double t = oy - m * pb.H;
          double d = std::sqrt(ox * ox + t * t);
          if (!(2.0 * rho_max <= mac * d)) {
            if (mlo > mhi) { mlo = m; mhi = m; }
            mlo = std::min(mlo, m);
            mhi = std::max(mhi, m);
          }
        }
        hp.root_off_mrange.push_back(mlo);
        hp.root_off_mrange.push_back(mhi);
      }
    }
  }

  // dual traversal for the explicit images
  hp.off_xy.clear();
  KeyHash oh;
  oh.xy = &hp.off_xy;
  std::vector<M2LEntry> m2l;
  std::vector<char> m2l_int;
  std::vector<NearEntry> nears;
  std::function<void(int, int, int, bool)> trav = [&](int D, int C, int m, bool interior) {
    const Cell& cd = hp.cells[D];
    const Cell& cc = hp.cells[C];
    double dx = cd.cx - cc.cx;
    double dy = cd.cy - cc.cy - m * pb.H;
    double d = std::sqrt(dx * dx + dy * dy);
    if (cd.rho + cc.rho <= mac * d) {
      m2l.push_back(M2LEntry{D, C, oh.get(dx, dy, scale), m});
      m2l_int.push_back(interior ? 1 : 0);
      return;
    }
    if (cd.leaf && cc.leaf) {
      nears.push_back(NearEntry{cd.leaf_index, C, m});
      return;
    }
    bool split_src = cd.leaf || (!cc.leaf && cc.rho >= cd.rho);
    if (split_src) {
      for (int k = 0; k < cc.n_child; ++k) trav(D, cc.first_child + k, m, interior);
    } else {
      for (int k = 0; k < cd.n_child; ++k) trav(cd.first_child + k, C, m, interior);
    }
  };
  hp.m_min = 0;
  hp.m_max = 0;
  for (int i = 0; i < M; ++i) {
    for (int j = 0; j < M; ++j) {
      int id = hp.root_pair_off[(size_t)i * M + j];
      int mlo = hp.root_off_mrange[2 * id], mhi = hp.root_off_mrange[2 * id + 1];
      for (int m = mlo; m <= mhi; ++m) {
        hp.m_min = std::min(hp.m_min, m);
        hp.m_max = std::max(hp.m_max, m);
        // a fibre's own image-0 block applied by FFT is not in the tree
        if (pb.self_fft && i == j && m == 0) continue;
        trav(hp.root_of_fibre[i], hp.root_of_fibre[j], m, i == j && m == 0);
      }
    }
  }

  // CSR by target
  auto csr = [&](int n_tgt, const std::vector<int>& tgt, std::vector<int>& ptr, std::vector<int>& perm) {
    ptr.assign(n_tgt + 1, 0);
    for (int t : tgt) ptr[t + 1]++;
    for (int i = 0; i < n_tgt; ++i) ptr[i + 1] += ptr[i];
    std::vector<int> pos(ptr.begin(), ptr.end() - 1);
    perm.assign(tgt.size(), 0);
    for (size_t e = 0; e < tgt.size(); ++e) perm[pos[tgt[e]]++] = (int)e;
  };
  {
    std::vector<int> tgt, perm;
    for (auto& e : m2l) tgt.push_back(e.tgt);
    csr(nc, tgt, hp.m2l_ptr, perm);
    hp.m2l_src.resize(perm.size());
    hp.m2l_off.resize(perm.size());
    hp.m2l_m.resize(perm.size());
    for (size_t i = 0; i < perm.size(); ++i) {
      hp.m2l_src[i] = m2l[perm[i]].src;
      hp.m2l_off[i] = m2l[perm[i]].off;
      hp.m2l_m[i] = m2l[perm[i]].m;
    }
    std::vector<int> tgti, permi, idx;
    for (size_t e = 0; e < m2l.size(); ++e)
      if (m2l_int[e]) { tgti.push_back(m2l[e].tgt); idx.push_back((int)e); }
    csr(nc, tgti, hp.m2li_ptr, permi);
    hp.m2li_src.resize(permi.size());
    hp.m2li_off.resize(permi.size());
    for (size_t i = 0; i < permi.size(); ++i) {
      hp.m2li_src[i] = m2l[idx[permi[i]]].src;
      hp.m2li_off[i] = m2l[idx[permi[i]]].off;
    }
  }
  {
    std::vector<int> tgt, perm;
    for (auto& e : nears) tgt.push_back(e.tgt_leaf);
    csr((int)hp.leaves.size(), tgt, hp.near_ptr, perm);
    hp.near_src.resize(perm.size());
    hp.near_m.resize(perm.size());
    hp.near_blk.resize(perm.size());
    hp.near_tgt.resize(perm.size());
    long long off = 0;
    for (size_t i = 0; i < perm.size(); ++i) {
      const NearEntry& e = nears[perm[i]];
      hp.near_src[i] = e.src;
      hp.near_m[i] = e.m;
      hp.near_blk[i] = off;
      hp.near_tgt[i] = e.tgt_leaf;
      const Cell& D = hp.cells[hp.leaves[e.tgt_leaf]];
      const Cell& C = hp.cells[e.src];
      off += (long long)(D.eend - D.ebeg) * (C.eend - C.ebeg);
    }
    hp.n_near_entries = off;
  }
  return true;
}

}  // namespace pfm
