// Host check of the nested-dissection plan tables that the HIP kernels index.
//
// Builds the plan of one geometry, or the combined plan of a batch, with the
// library's own planner (plan.cpp) and verifies every range a kernel forms an
// address from: front arena blocks, solve-vector slots, global indices,
// boundary-to-parent maps, pivot-permutation and diagonal-block-inverse
// slots, inverse work slots, the gather index of children's boundary rows,
// and the assembly blocks.  Ranges that must not overlap are checked for
// overlap.  Small plans also check that every entry of P is assembled
// exactly once.
//
// usage: plan_check [-s] [-p] [-v] [-c NC] d,n,b,order [d,n,b,order ...]
//        (several: one batch; -s: streamed storage, see layout_plan; -p: point
//        stencil pattern, see build_plan; -v: print the levels; -c: NC
//        unknowns per grid point, see expand_plan)
// Prints "ok ..." and exits 0, or prints the first violation and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "plan.hpp"

using namespace spp;

namespace {

int fail(const std::string& m) {
  std::printf("FAIL %s\n", m.c_str());
  return 1;
}

// [a, a + len) ranges: all inside [0, limit) and pairwise disjoint.
bool disjoint(std::vector<std::pair<int64_t, int64_t>> r, int64_t limit, std::string& why) {
  std::sort(r.begin(), r.end());
  int64_t end = 0;
  for (const auto& x : r) {
    if (x.second == 0) continue;
    if (x.first < 0 || x.first + x.second > limit) {
      why = "range [" + std::to_string(x.first) + ", " + std::to_string(x.first + x.second) + ") outside " +
            std::to_string(limit);
      return false;
    }
    if (x.first < end) {
      why = "ranges overlap at " + std::to_string(x.first);
      return false;
    }
    end = x.first + x.second;
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  int first = 1, storage = 0, pattern = 0, nc = 1;
  bool verbose = false;
  while (first < argc && argv[first][0] == '-') {
    const std::string o = argv[first++];
    if (o == "-s") storage = 1;
    else if (o == "-p") pattern = 1;
    else if (o == "-v") verbose = true;
    else if (o == "-c" && first < argc) nc = std::atoi(argv[first++]);
    else return fail("unknown option " + o);
  }
  if (argc <= first) return fail("no geometry given");
  std::vector<Plan> plans(argc - first);
  std::vector<int64_t> Ns;
  for (int a = first; a < argc; ++a) {
    int d, n, b, order;
    if (std::sscanf(argv[a], "%d,%d,%d,%d", &d, &n, &b, &order) != 4) return fail("bad geometry " + std::string(argv[a]));
    std::string err = build_plan(d, n, b, order, plans[a - first], pattern);
    if (!err.empty()) return fail("build_plan: " + err);
    err = expand_plan(plans[a - first], nc);
    if (!err.empty()) return fail("expand_plan: " + err);
    Ns.push_back(plans[a - first].N * nc);   // unknowns
  }
  Plan P;
  std::vector<int> inst;
  if (plans.size() == 1) {
    P = plans[0];
    inst.assign(P.fronts.size(), 0);
  } else {
    std::vector<const Plan*> raw;
    for (const Plan& p : plans) raw.push_back(&p);
    std::string err = combine_plans(raw, P, inst);
    if (!err.empty()) return fail("combine_plans: " + err);
  }
  layout_plan(P, storage);
  PlanTables T;
  {
    std::string err = build_tables(P, inst, T);
    if (!err.empty()) return fail("build_tables: " + err);
  }
  const int nf = static_cast<int>(P.fronts.size());
  std::string why;

  // Levels cover the fronts and the assembly blocks in order.
  int fexp = 0, bexp = 0;
  for (size_t l = 0; l < P.levels.size(); ++l) {
    const Level& L = P.levels[l];
    if (L.begin != fexp || L.end < L.begin) return fail("level front range " + std::to_string(l));
    if (L.blk_begin != bexp || L.blk_end < L.blk_begin) return fail("level block range " + std::to_string(l));
    fexp = L.end;
    bexp = L.blk_end;
    int mF = 0, mP = 0, mK = 0, mC = 0;
    for (int fi = L.begin; fi < L.end; ++fi) {
      const Front& f = P.fronts[fi];
      mF = std::max(mF, f.F); mP = std::max(mP, f.p); mK = std::max(mK, f.F - f.p);
      mC = std::max<int>(mC, static_cast<int>(f.children.size()));
    }
    if (mF != L.maxF || mP != L.maxP || mK != L.maxK || mC != L.max_children)
      return fail("level maxima " + std::to_string(l));
    if (mC > 8) return fail("more than 8 children");
    for (int bi = L.blk_begin; bi < L.blk_end; ++bi)
      if (P.blocks[bi].front < L.begin || P.blocks[bi].front >= L.end) return fail("block outside its level");
  }
  if (fexp != nf || bexp != static_cast<int>(P.blocks.size())) return fail("levels do not cover the plan");

  // Fronts: sizes, arena and vector slots, indices.
  std::vector<std::pair<int64_t, int64_t>> arena, vec, perm, dblk;
  std::vector<std::vector<int>> owner(Ns.size());
  for (size_t i = 0; i < Ns.size(); ++i) owner[i].assign(Ns[i], -1);
  for (int fi = 0; fi < nf; ++fi) {
    const Front& f = P.fronts[fi];
    const FrontTable& t = T.fronts[fi];
    if (f.p < 1 || f.F < f.p) return fail("front sizes " + std::to_string(fi));
    if (t.F != f.F || t.p != f.p || t.off != f.off || t.voff != f.voff || t.idx != f.idx || t.map != f.map)
      return fail("table copy of front " + std::to_string(fi));
    arena.emplace_back(f.off, static_cast<int64_t>(f.F) * f.F);
    vec.emplace_back(f.voff, f.F);
    perm.emplace_back(t.perm, f.p);
    dblk.emplace_back(t.dblk, (f.p + 31) / 32);
    // the diagonal-block kernels address slot dblk + k0 / 32 for k0 < p
    if (t.dblk + (f.p - 1) / 32 >= T.dblk_total) return fail("diagonal-block slot past dinv, front " + std::to_string(fi));
    if (f.idx < 0 || f.idx + f.F > static_cast<int64_t>(P.idx.size())) return fail("idx range " + std::to_string(fi));
    const int64_t N = Ns[t.inst];
    std::set<int> seen;
    for (int k = 0; k < f.F; ++k) {
      const int g = P.idx[f.idx + k];
      if (g < 0 || g >= N) return fail("global index out of the grid, front " + std::to_string(fi));
      if (!seen.insert(g).second) return fail("repeated point in front " + std::to_string(fi));
      if (k < f.p) {
        if (owner[t.inst][g] >= 0) return fail("point eliminated twice");
        owner[t.inst][g] = fi;
      }
    }
  }
  for (size_t i = 0; i < Ns.size(); ++i)
    for (int64_t g = 0; g < Ns[i]; ++g)
      if (owner[i][g] < 0) return fail("point never eliminated");
  if (storage == 0) {
    if (!disjoint(arena, P.arena_elems, why)) return fail("front arena: " + why);
    for (const Front& f : P.fronts)
      if (f.foff != f.off || f.uoff != f.off + (int64_t)f.p * f.F || f.ldu != f.F) return fail("resident factor offsets");
  } else {
    // Each level's fronts lie in its own arena range, disjoint from the
    // level below (whose Schur complements it adds); factors are compact.
    for (size_t l = 0; l < P.levels.size(); ++l) {
      std::vector<std::pair<int64_t, int64_t>> two;
      for (size_t m = (l ? l - 1 : 0); m <= l; ++m) {
        const Level& L = P.levels[m];
        for (int fi = L.begin; fi < L.end; ++fi) {
          const Front& f = P.fronts[fi];
          if (f.off < L.arena_lo || f.off + (int64_t)f.F * f.F > L.arena_hi) return fail("front outside its level range");
          two.emplace_back(f.off, (int64_t)f.F * f.F);
        }
      }
      if (!disjoint(two, P.arena_elems, why)) return fail("levels " + std::to_string(l) + " and below: " + why);
    }
    std::vector<std::pair<int64_t, int64_t>> fac;
    for (const Front& f : P.fronts) {
      if (f.ldu != f.p || f.uoff != f.foff + (int64_t)f.p * f.F) return fail("streamed factor offsets");
      fac.emplace_back(f.foff, (int64_t)f.p * f.F);
      fac.emplace_back(f.uoff, (int64_t)f.p * (f.F - f.p));
    }
    if (!disjoint(fac, P.fstore_elems, why)) return fail("factor store: " + why);
  }
  if (!disjoint(vec, P.vec_elems, why)) return fail("vector arena: " + why);
  if (!disjoint(perm, T.perm_total, why)) return fail("pivot permutation slots: " + why);
  if (!disjoint(dblk, T.dblk_total, why)) return fail("diagonal-block slots: " + why);

  // Inverse work slots: disjoint within each level, inside the work buffer.
  for (const Level& L : P.levels) {
    std::vector<std::pair<int64_t, int64_t>> xw;
    for (int fi = L.begin; fi < L.end; ++fi) xw.emplace_back(T.fronts[fi].xoff, 2LL * P.fronts[fi].p * P.fronts[fi].F);
    if (!disjoint(xw, T.xwork_elems, why)) return fail("inverse work slots: " + why);
  }

  // Parents, children and boundary maps.
  for (int fi = 0; fi < nf; ++fi) {
    const Front& f = P.fronts[fi];
    const FrontTable& t = T.fronts[fi];
    for (int c = 0; c < t.nchild; ++c) {
      if (t.child[c] < 0 || t.child[c] >= fi) return fail("child index of front " + std::to_string(fi));
      if (T.fronts[t.child[c]].parent != fi) return fail("child's parent link");
      if (T.fronts[t.child[c]].inst != t.inst) return fail("child of another problem");
    }
    if (t.parent < 0) {
      if (f.F != f.p) return fail("root with boundary points");
      continue;
    }
    const Front& par = P.fronts[t.parent];
    if (f.map < 0 || f.map + (f.F - f.p) > static_cast<int64_t>(P.map.size())) return fail("map range");
    std::set<int> seen;
    for (int k = 0; k < f.F - f.p; ++k) {
      const int ps = P.map[f.map + k];
      if (ps < 0 || ps >= par.F) return fail("map value outside the parent, front " + std::to_string(fi));
      if (!seen.insert(ps).second) return fail("two boundary points on one parent position");
      if (P.idx[par.idx + ps] != P.idx[f.idx + f.p + k]) return fail("map points at another grid point");
    }
  }

  // Gather index of the children's boundary rows.
  for (int fi = 0; fi < nf; ++fi) {
    const Front& f = P.fronts[fi];
    const FrontTable& t = T.fronts[fi];
    if (t.gptr < 0 || t.gptr + f.F >= static_cast<int64_t>(T.gptr.size())) return fail("gptr range");
    for (int i = 0; i < f.F; ++i) {
      const int a = T.gptr[t.gptr + i], b = T.gptr[t.gptr + i + 1];
      if (a < 0 || b < a || b > static_cast<int64_t>(T.gsrc.size())) return fail("gptr offsets");
      for (int e = a; e < b; ++e) {
        const int64_t src = T.gsrc[e];
        bool ok = false;
        for (int c = 0; c < t.nchild && !ok; ++c) {
          const Front& ch = P.fronts[t.child[c]];
          ok = src >= ch.voff + ch.p && src < ch.voff + ch.F;
        }
        if (!ok) return fail("gathered row outside the children's boundary slots, front " + std::to_string(fi));
      }
    }
  }

  // Assembly blocks.
  const bool small = P.N <= 70000;
  std::set<std::pair<int64_t, int64_t>> entries;
  for (size_t bi = 0; bi < P.blocks.size(); ++bi) {
    const AsmBlock& B = P.blocks[bi];
    if (B.front < 0 || B.front >= nf) return fail("block front");
    const Front& f = P.fronts[B.front];
    const Plan& own = plans[T.fronts[B.front].inst];
    if (B.type < 0 || B.type >= static_cast<int>(own.types.size())) return fail("block set type");
    const SetType& ST = own.types[B.type];
    const int nS = ST.nS * own.nc, nG = ST.nG * own.nc;   // unknowns of the set lists
    int64_t anchors = 1;
    for (int i = 0; i < own.d; ++i) anchors *= own.n / own.bs;
    if (B.anchor < 0 || B.anchor >= anchors) return fail("block anchor");
    if (B.rowpos < 0 || B.rowpos + nS > static_cast<int64_t>(P.pos.size())) return fail("block row positions");
    if (B.colpos < 0 || B.colpos + nG > static_cast<int64_t>(P.pos.size())) return fail("block column positions");
    bool full = true;
    for (int i = 0; i < nS; ++i) {
      const int r = P.pos[B.rowpos + i];
      if (r < 0 || r >= f.F) return fail("block row position outside the front");
      if (i == 0) full = r < f.p;
      if ((r < f.p) != full) return fail("block mixes pivot and boundary rows");
    }
    for (int j = 0; j < nG; ++j) {
      const int c = P.pos[B.colpos + j];
      if (c < -1 || c >= f.F) return fail("block column position outside the front");
      if (!full && c >= f.p) return fail("boundary rows assembled outside the pivot columns");
    }
    if (small) {
      for (int i = 0; i < nS; ++i)
        for (int j = 0; j < nG; ++j) {
          const int c = P.pos[B.colpos + j];
          if (c < 0) continue;
          const int64_t gr = P.idx[f.idx + P.pos[B.rowpos + i]], gc = P.idx[f.idx + c];
          const int64_t key = static_cast<int64_t>(T.fronts[B.front].inst) << 40;
          if (!entries.insert({key + gr, gc}).second) return fail("an entry of P assembled twice");
        }
    }
  }
  int64_t fmax = 0;
  for (const Front& f : P.fronts) fmax = std::max<int64_t>(fmax, f.F);
  if (verbose)
    for (size_t l = 0; l < P.levels.size(); ++l) {
      const Level& L = P.levels[l];
      std::printf("level %zu: %d fronts, max F %d, max p %d\n", l, L.end - L.begin, L.maxF, L.maxP);
    }
  std::printf("ok fronts %d levels %zu max_front %lld arena %lld store %lld vec %lld dinv_slots %d blocks %zu%s\n",
              nf, P.levels.size(), (long long)fmax, (long long)P.arena_elems, (long long)P.fstore_elems,
              (long long)P.vec_elems, T.dblk_total, P.blocks.size(), small ? " (P entries checked)" : "");
  return 0;
}
