// Nested-dissection plan construction (host).  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <sstream>

namespace spp {

namespace {

int64_t ipow(int64_t a, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= a;
  return r;
}

// Box widths per level, leaves first.
std::vector<std::vector<int>> level_shapes(int d, int n, int b, int order) {
  std::vector<std::vector<int>> shapes;
  std::vector<int> w(d, b);
  shapes.push_back(w);
  if (order == 0) {
    while (w[0] < n) {
      for (int i = 0; i < d; ++i) w[i] *= 2;
      shapes.push_back(w);
    }
  } else {
    int axis = 0;
    for (;;) {
      bool done = true;
      for (int i = 0; i < d; ++i) done = done && (w[i] >= n);
      if (done) break;
      while (w[axis] >= n) axis = (axis + 1) % d;
      w[axis] *= 2;
      shapes.push_back(w);
      axis = (axis + 1) % d;
    }
  }
  return shapes;
}

SetType make_type(int d, int b, int mask) {
  SetType t;
  t.mask = mask;
  std::vector<int> lo(d), hi(d);
  for (int i = 0; i < d; ++i) {
    bool pinned = (mask >> i) & 1;
    lo[i] = pinned ? -1 : 0;
    hi[i] = pinned ? 1 : b;
  }
  auto in_S = [&](const std::vector<int>& o) {
    for (int i = 0; i < d; ++i) {
      bool pinned = (mask >> i) & 1;
      if (pinned ? (o[i] != 0) : (o[i] < 1 || o[i] > b - 1)) return false;
    }
    return true;
  };
  std::vector<int> S, B;
  std::vector<int> o(lo);
  for (;;) {
    std::vector<int>& dst = in_S(o) ? S : B;
    dst.insert(dst.end(), o.begin(), o.end());
    int i = d - 1;
    while (i >= 0 && o[i] == hi[i]) { o[i] = lo[i]; --i; }
    if (i < 0) break;
    ++o[i];
  }
  t.nS = static_cast<int>(S.size()) / d;
  if (t.nS == 0) return t;   // a set type with no points (boxes of width 1)
  t.nB = static_cast<int>(B.size()) / d;
  t.nG = t.nS + t.nB;
  t.off = S;
  t.off.insert(t.off.end(), B.begin(), B.end());
  return t;
}

}  // namespace

std::string validate_grid(int d, int n, int b) {
  if (d != 2 && d != 3) return "dim must be 2 or 3";
  if (n < 4 || (n & 1)) return "n must be even and >= 4";
  if (b < 2 || n % b) return "b must be >= 2 and divide n";
  const int m = n / b;
  if (m < 2 || (m & (m - 1))) return "n / b must be a power of two >= 2";
  return std::string();
}

std::string build_plan(int d, int n, int b, int order, Plan& P, int pattern) {
  std::ostringstream err;
  {
    std::string v = validate_grid(d, n, b);
    if (!v.empty()) return v;
  }
  if (pattern != 0 && pattern != 1) return "pattern must be 0 (sets) or 1 (points)";
  // The stencil sets partition the grid by boxes of width bs: the leaf
  // boxes (b), or single points (bs = 1: every point its own set).
  const int bs = pattern == 1 ? 1 : b;
  const int m = n / bs;
  P = Plan();
  P.d = d; P.n = n; P.b = b; P.m = n / b; P.order = order;
  P.pattern = pattern; P.bs = bs;
  P.N = ipow(n, d);
  const int64_t N = P.N;
  const int ntypes = 1 << d;
  const int64_t nanchor = ipow(m, d);
  for (int t = 0; t < ntypes; ++t) P.types.push_back(make_type(d, bs, t));

  std::vector<int> owner(N, -1), posmap(N, -1);
  std::vector<int> set_stamp(static_cast<size_t>(ntypes * nanchor), -1);
  std::vector<std::vector<int>> front_lo;
  auto shapes = level_shapes(d, n, b, order);

  std::vector<int> coord(d), crd(d);
  auto ravel = [&](const std::vector<int>& x) {
    int64_t g = 0;
    for (int i = 0; i < d; ++i) g = g * n + x[i];
    return g;
  };
  auto set_of = [&](int64_t g, int& type, int& anchor) {
    int64_t r = g;
    int msk = 0;
    int64_t an = 0, mul = 1;
    for (int i = d - 1; i >= 0; --i) {
      int x = static_cast<int>(r % n);
      r /= n;
      if (x % bs == 0) msk |= 1 << i;
      an += mul * (x / bs);
      mul *= m;
    }
    type = msk;
    anchor = static_cast<int>(an);
  };
  // Global index of offset `o` of a set anchored at box `anchor`.
  auto point_of = [&](int anchor, const int* o) {
    int64_t g = 0;
    int64_t a = anchor;
    std::vector<int> ac(d);
    for (int i = d - 1; i >= 0; --i) { ac[i] = static_cast<int>(a % m); a /= m; }
    for (int i = 0; i < d; ++i) g = g * n + ((ac[i] * bs + o[i]) % n + n) % n;
    return g;
  };

  for (size_t lv = 0; lv < shapes.size(); ++lv) {
    const std::vector<int>& w = shapes[lv];
    Level L;
    L.begin = static_cast<int>(P.fronts.size());
    L.blk_begin = static_cast<int>(P.blocks.size());
    std::vector<int> nbox(d);
    int64_t boxes = 1;
    for (int i = 0; i < d; ++i) { nbox[i] = n / w[i]; boxes *= nbox[i]; }
    for (int64_t bx = 0; bx < boxes; ++bx) {
      std::vector<int> lo(d), len(d);
      int64_t r = bx;
      for (int i = d - 1; i >= 0; --i) {
        int bi = static_cast<int>(r % nbox[i]);
        r /= nbox[i];
        bool full = (w[i] == n);
        lo[i] = full ? 0 : bi * w[i];
        len[i] = full ? n : w[i] + 1;
      }
      std::vector<int> piv, bnd;
      std::vector<int> u(d, 0);
      for (;;) {
        bool interior = true;
        for (int i = 0; i < d; ++i) {
          int ui = lo[i] + u[i];
          crd[i] = ui % n;
          if (w[i] != n && (u[i] == 0 || u[i] == len[i] - 1)) interior = false;
        }
        int64_t g = ravel(crd);
        if (owner[g] < 0) (interior ? piv : bnd).push_back(static_cast<int>(g));
        int i = d - 1;
        while (i >= 0 && u[i] == len[i] - 1) { u[i] = 0; --i; }
        if (i < 0) break;
        ++u[i];
      }
      if (piv.empty()) {
        err << "box " << bx << " at level " << lv << " has no pivots";
        return err.str();
      }
      Front f;
      f.level = static_cast<int>(lv);
      f.p = static_cast<int>(piv.size());
      f.F = f.p + static_cast<int>(bnd.size());
      f.idx = static_cast<int>(P.idx.size());
      int fid = static_cast<int>(P.fronts.size());
      P.idx.insert(P.idx.end(), piv.begin(), piv.end());
      P.idx.insert(P.idx.end(), bnd.begin(), bnd.end());
      for (int g : piv) owner[g] = fid;
      for (int k = 0; k < f.F; ++k) posmap[P.idx[f.idx + k]] = k;

      // Assembly blocks: block rows of the sets eliminated here (all their
      // columns still alive), then block rows of boundary sets restricted to
      // this front's pivot columns.  Each entry of P is assembled exactly once,
      // into the front that eliminates its row or its column first.
      std::vector<int> piv_sets;
      for (int g : piv) {
        int ty, an;
        set_of(g, ty, an);
        size_t sid = static_cast<size_t>(ty) * nanchor + an;
        if (set_stamp[sid] != fid) { set_stamp[sid] = fid; piv_sets.push_back(static_cast<int>(sid)); }
      }
      auto emit = [&](int sid, bool full_rows) -> bool {
        int ty = static_cast<int>(sid / nanchor), an = static_cast<int>(sid % nanchor);
        const SetType& T = P.types[ty];
        AsmBlock blk;
        blk.front = fid; blk.type = ty; blk.anchor = an;
        blk.rowpos = static_cast<int>(P.pos.size());
        for (int i = 0; i < T.nS; ++i) {
          int64_t g = point_of(an, &T.off[i * d]);
          int ps = posmap[g];
          if (ps < 0 || (full_rows ? ps >= f.p : ps < f.p)) return false;
          P.pos.push_back(ps);
        }
        blk.colpos = static_cast<int>(P.pos.size());
        for (int j = 0; j < T.nG; ++j) {
          int64_t g = point_of(an, &T.off[j * d]);
          int ps;
          if (full_rows) {
            ps = (owner[g] < 0 || owner[g] == fid) ? posmap[g] : -1;
            if ((owner[g] < 0 || owner[g] == fid) && ps < 0) return false;
          } else {
            ps = (owner[g] == fid) ? posmap[g] : -1;
          }
          P.pos.push_back(ps);
        }
        P.blocks.push_back(blk);
        return true;
      };
      for (int sid : piv_sets) {
        if (!emit(sid, true)) { err << "pivot set outside front " << fid; return err.str(); }
      }
      for (int g : piv) {
        int64_t rr = g;
        for (int i = d - 1; i >= 0; --i) { coord[i] = static_cast<int>(rr % n); rr /= n; }
        for (int nb3 = 0; nb3 < ipow(3, d); ++nb3) {
          int t = nb3;
          for (int i = d - 1; i >= 0; --i) { crd[i] = ((coord[i] + t % 3 - 1) % n + n) % n; t /= 3; }
          int64_t g2 = ravel(crd);
          if (owner[g2] >= 0) continue;  // row already eliminated: assembled there
          int ty, an;
          set_of(g2, ty, an);
          size_t sid = static_cast<size_t>(ty) * nanchor + an;
          if (set_stamp[sid] == fid) continue;
          set_stamp[sid] = fid;
          if (!emit(static_cast<int>(sid), false)) {
            err << "boundary set of front " << fid << " not on its surface";
            return err.str();
          }
        }
      }
      for (int k = 0; k < f.F; ++k) posmap[P.idx[f.idx + k]] = -1;
      front_lo.push_back(lo);
      P.fronts.push_back(f);
      L.maxF = std::max(L.maxF, f.F);
      L.maxP = std::max(L.maxP, f.p);
      L.maxK = std::max(L.maxK, f.F - f.p);
    }
    L.end = static_cast<int>(P.fronts.size());
    L.blk_end = static_cast<int>(P.blocks.size());
    P.levels.push_back(L);
  }
  for (int64_t g = 0; g < N; ++g)
    if (owner[g] < 0) return "ordering left a point uneliminated";

  // Parent links, child slots, boundary -> parent position maps.
  for (size_t lv = 0; lv + 1 < P.levels.size(); ++lv) {
    const std::vector<int>& W = shapes[lv + 1];
    std::vector<int> nbox(d);
    for (int i = 0; i < d; ++i) nbox[i] = n / W[i];
    for (int fi = P.levels[lv].begin; fi < P.levels[lv].end; ++fi) {
      int64_t pb = 0;
      for (int i = 0; i < d; ++i) pb = pb * nbox[i] + (W[i] == n ? 0 : front_lo[fi][i] / W[i]);
      int parent = P.levels[lv + 1].begin + static_cast<int>(pb);
      Front& c = P.fronts[fi];
      c.parent = parent;
      c.slot = static_cast<int>(P.fronts[parent].children.size());
      P.fronts[parent].children.push_back(fi);
    }
  }
  for (auto& L : P.levels) {
    for (int fi = L.begin; fi < L.end; ++fi)
      L.max_children = std::max<int>(L.max_children, static_cast<int>(P.fronts[fi].children.size()));
  }
  for (size_t fi = 0; fi < P.fronts.size(); ++fi) {
    Front& c = P.fronts[fi];
    c.map = static_cast<int>(P.map.size());
    if (c.parent < 0) {
      if (c.F != c.p) return "root front has boundary points";
      continue;
    }
    const Front& par = P.fronts[c.parent];
    for (int k = 0; k < par.F; ++k) posmap[P.idx[par.idx + k]] = k;
    for (int k = c.p; k < c.F; ++k) {
      int ps = posmap[P.idx[c.idx + k]];
      if (ps < 0) { err << "front " << fi << " boundary point missing from parent"; return err.str(); }
      P.map.push_back(ps);
    }
    for (int k = 0; k < par.F; ++k) posmap[P.idx[par.idx + k]] = -1;
  }

  layout_plan(P, 0);
  return std::string();
}

std::string expand_plan(Plan& P, int nc) {
  if (nc < 1 || nc > 3) return "unknowns per point must be 1, 2 or 3";
  if (P.nc != 1) return "plan already expanded";
  if (nc == 1) return std::string();
  const int64_t N = P.N;
  if ((int64_t)nc * N > INT32_MAX) return "grid too large for vector unknowns";
  auto widen = [&](const std::vector<int>& src, int64_t b, int64_t cnt, std::vector<int>& dst, bool global) {
    for (int64_t k = 0; k < cnt; ++k) {
      const int v = src[b + k];
      for (int c = 0; c < nc; ++c)
        dst.push_back(v < 0 ? -1 : global ? static_cast<int>(c * N + v) : v * nc + c);
    }
  };
  std::vector<int> idx, map, pos;
  idx.reserve(P.idx.size() * nc);
  map.reserve(P.map.size() * nc);
  pos.reserve(P.pos.size() * nc);
  for (Front& f : P.fronts) {
    const int i0 = static_cast<int>(idx.size()), m0 = static_cast<int>(map.size());
    widen(P.idx, f.idx, f.F, idx, true);
    if (f.parent >= 0) widen(P.map, f.map, f.F - f.p, map, false);
    f.idx = i0;
    f.map = m0;
    f.F *= nc;
    f.p *= nc;
  }
  for (AsmBlock& B : P.blocks) {
    const SetType& T = P.types[B.type];
    if (B.rowpos >= 0) {
      const int r0 = static_cast<int>(pos.size());
      widen(P.pos, B.rowpos, T.nS, pos, false);
      B.rowpos = r0;
    }
    if (B.colpos >= 0) {
      const int c0 = static_cast<int>(pos.size());
      widen(P.pos, B.colpos, T.nG, pos, false);
      B.colpos = c0;
    }
  }
  for (Level& L : P.levels) {
    L.maxF *= nc;
    L.maxP *= nc;
    L.maxK *= nc;
  }
  P.idx.swap(idx);
  P.map.swap(map);
  P.pos.swap(pos);
  P.nc = nc;
  layout_plan(P, 0);
  return std::string();
}

std::string combine_plans(const std::vector<const Plan*>& plans, Plan& out, std::vector<int>& front_inst) {
  if (plans.empty()) return "empty batch";
  out = Plan();
  front_inst.clear();
  const Plan& p0 = *plans[0];
  out.d = p0.d; out.n = p0.n; out.b = p0.b; out.m = p0.m; out.order = p0.order;
  out.types = p0.types;
  size_t nlev = 0;
  for (const Plan* P : plans) {
    if (P->d != p0.d) return "all problems of a batch must have the same dimension";
    nlev = std::max(nlev, P->levels.size());
    out.N += P->N;
  }
  const size_t ni = plans.size();
  std::vector<std::vector<int>> newid(ni);
  std::vector<int> idx_base(ni), map_base(ni), pos_base(ni);
  for (size_t i = 0; i < ni; ++i) {
    newid[i].assign(plans[i]->fronts.size(), -1);
    idx_base[i] = static_cast<int>(out.idx.size());
    out.idx.insert(out.idx.end(), plans[i]->idx.begin(), plans[i]->idx.end());
    map_base[i] = static_cast<int>(out.map.size());
    out.map.insert(out.map.end(), plans[i]->map.begin(), plans[i]->map.end());
    pos_base[i] = static_cast<int>(out.pos.size());
    out.pos.insert(out.pos.end(), plans[i]->pos.begin(), plans[i]->pos.end());
  }
  for (size_t l = 0; l < nlev; ++l) {
    Level L;
    L.begin = static_cast<int>(out.fronts.size());
    L.blk_begin = static_cast<int>(out.blocks.size());
    for (size_t i = 0; i < ni; ++i) {
      const Plan& P = *plans[i];
      if (l >= P.levels.size()) continue;
      const Level& PL = P.levels[l];
      for (int fi = PL.begin; fi < PL.end; ++fi) {
        Front f = P.fronts[fi];
        f.level = static_cast<int>(l);
        f.idx += idx_base[i];
        f.map += map_base[i];
        for (int& c : f.children) {
          c = newid[i][c];
          if (c < 0) return "child front of a batch problem placed after its parent";
        }
        f.parent = -1;
        newid[i][fi] = static_cast<int>(out.fronts.size());
        out.fronts.push_back(f);
        front_inst.push_back(static_cast<int>(i));
        L.maxF = std::max(L.maxF, f.F);
        L.maxP = std::max(L.maxP, f.p);
        L.maxK = std::max(L.maxK, f.F - f.p);
        L.max_children = std::max<int>(L.max_children, static_cast<int>(f.children.size()));
      }
      for (int bi = PL.blk_begin; bi < PL.blk_end; ++bi) {
        AsmBlock B = P.blocks[bi];
        B.front = newid[i][B.front];
        if (B.rowpos >= 0) B.rowpos += pos_base[i];
        if (B.colpos >= 0) B.colpos += pos_base[i];
        out.blocks.push_back(B);
      }
    }
    L.end = static_cast<int>(out.fronts.size());
    L.blk_end = static_cast<int>(out.blocks.size());
    out.levels.push_back(L);
  }
  layout_plan(out, 0);
  return std::string();
}

void layout_plan(Plan& P, int storage) {
  auto pad = [](int64_t e) { return (e + 15) / 16 * 16; };
  P.storage = storage;
  P.factor_entries = 0;
  P.factor_flops = 0;
  P.max_front = 0;
  int64_t voff = 0;
  for (Front& f : P.fronts) {
    f.voff = voff;
    voff += pad(f.F);
    const double p = f.p, k = f.F - f.p;
    P.factor_entries += static_cast<int64_t>(f.p) * f.p + 2LL * f.p * (f.F - f.p);
    P.factor_flops += 8.0 * (p * p * p / 3.0 + p * p * k + p * k * k);
    P.max_front = std::max(P.max_front, f.F);
  }
  P.vec_elems = voff;
  const size_t nl = P.levels.size();
  std::vector<int64_t> S(nl, 0);
  for (size_t l = 0; l < nl; ++l)
    for (int fi = P.levels[l].begin; fi < P.levels[l].end; ++fi)
      S[l] += pad(static_cast<int64_t>(P.fronts[fi].F) * P.fronts[fi].F);
  int64_t A = 0;
  if (storage == 0) {
    for (size_t l = 0; l < nl; ++l) A += S[l];
  } else {
    for (size_t l = 0; l < nl; ++l) A = std::max(A, S[l] + (l ? S[l - 1] : 0));
  }
  int64_t off = 0, fo = 0;
  for (size_t l = 0; l < nl; ++l) {
    Level& L = P.levels[l];
    if (storage == 1) off = (l % 2 == 0) ? 0 : A - S[l];
    L.arena_lo = off;
    for (int fi = L.begin; fi < L.end; ++fi) {
      Front& f = P.fronts[fi];
      f.off = off;
      off += pad(static_cast<int64_t>(f.F) * f.F);
      if (storage == 0) {
        f.foff = f.off;
        f.uoff = f.off + static_cast<int64_t>(f.p) * f.F;
        f.ldu = f.F;
      } else {
        f.foff = fo;
        f.uoff = fo + static_cast<int64_t>(f.p) * f.F;
        f.ldu = f.p;
        fo += pad(static_cast<int64_t>(f.p) * f.F + static_cast<int64_t>(f.p) * (f.F - f.p));
      }
    }
    L.arena_hi = off;
  }
  P.arena_elems = A;
  P.fstore_elems = fo;
}

std::string build_tables(const Plan& P, const std::vector<int>& front_inst, PlanTables& T) {
  T = PlanTables();
  if (front_inst.size() != P.fronts.size()) return "front_inst size mismatch";
  T.fronts.resize(P.fronts.size());
  std::vector<int> parent(P.fronts.size(), -1);
  for (size_t fi = 0; fi < P.fronts.size(); ++fi)
    for (int c : P.fronts[fi].children) parent[c] = static_cast<int>(fi);
  for (const Level& L : P.levels) {
    // Inverse work slots for every level (the precision decides which
    // levels use them): XL, XU (p x p each), then Lt, Ut ((F - p) x p each).
    int64_t xo = 0;
    double e0 = 0, e1 = 0, e2 = 0;
    std::vector<int> hF, hP;
    for (int fi = L.begin; fi < L.end; ++fi) {
      const Front& f = P.fronts[fi];
      FrontTable& g = T.fronts[fi];
      g.off = f.off; g.voff = f.voff; g.xoff = xo;
      g.foff = f.foff; g.uoff = f.uoff; g.ldu = f.ldu;
      g.F = f.F; g.p = f.p; g.idx = f.idx; g.map = f.map; g.perm = T.perm_total;
      g.dblk = T.dblk_total;
      g.inst = front_inst[fi];
      g.parent = parent[fi];
      T.dblk_total += (f.p + 31) / 32;
      g.nchild = static_cast<int>(f.children.size());
      if (g.nchild > 8) return "more than 8 children";
      for (int c = 0; c < g.nchild; ++c) g.child[c] = f.children[c];
      T.perm_total += f.p;
      xo += 2LL * f.p * f.F;
      e0 += 0.5 * f.p * (f.p - 1.0);
      e1 += 0.5 * f.p * (f.p + 1.0);
      e2 += (double)(f.F - f.p) * f.p;
      hF.push_back(f.F);
      hP.push_back(f.p);
    }
    T.level_ent.insert(T.level_ent.end(), {e0, e1, e2});
    T.level_F.push_back(hF);
    T.level_p.push_back(hP);
    T.xwork_elems = std::max(T.xwork_elems, xo);
  }
  // Children's boundary rows by parent position (counting sort, children in
  // order, so a position's sum keeps the order of the plain gather).
  for (size_t fi = 0; fi < P.fronts.size(); ++fi) {
    const Front& f = P.fronts[fi];
    T.fronts[fi].gptr = static_cast<int>(T.gptr.size());
    std::vector<int> cnt(f.F + 1, 0);
    for (int c : f.children) {
      const Front& ch = P.fronts[c];
      for (int jj = 0; jj < ch.F - ch.p; ++jj)
        if (P.map[ch.map + jj] >= 0) ++cnt[P.map[ch.map + jj] + 1];
    }
    for (int i = 0; i < f.F; ++i) cnt[i + 1] += cnt[i];
    const int64_t base = static_cast<int64_t>(T.gsrc.size());
    for (int i = 0; i <= f.F; ++i) T.gptr.push_back(static_cast<int>(base + cnt[i]));
    T.gsrc.resize(T.gsrc.size() + cnt[f.F]);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int c : f.children) {
      const Front& ch = P.fronts[c];
      for (int jj = 0; jj < ch.F - ch.p; ++jj)
        if (P.map[ch.map + jj] >= 0) T.gsrc[base + fill[P.map[ch.map + jj]]++] = ch.voff + ch.p + jj;
    }
    if (T.gsrc.size() > (size_t)INT32_MAX) return "plan too large";
  }
  return std::string();
}

}  // namespace spp
