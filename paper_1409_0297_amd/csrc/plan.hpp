// Host-side nested-dissection plan: set types, fronts, index maps.
//
// Geometry of Section 2.3: leaf boxes of width b with boundaries on the grid
// lines j_i = 0 (mod b); the leaf set partition into cells, faces, edges and
// vertices; gamma(S) = S widened by one grid step in every direction (mod n).
// Fronts follow the box hierarchy of Figure 1: a box eliminates the points of
// its open interior that its sub-boxes left, against the remaining points on
// its surface.  Boxes merge 2^d at a time (octree) or 2 at a time along the
// axes in turn (bisection); the last box is the whole periodic domain.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace spp {

// One orientation-resolved set type.  Bit i of `mask` set means axis i is
// pinned to a leaf box face (cell: 0, vertex: 2^d - 1).
struct SetType {
  int mask = 0;
  int nS = 0, nB = 0, nG = 0;   // |S|, |beta(S)|, |gamma(S)| = nS + nB
  // Grid offsets from the leaf box corner (a_0 b, ..., a_{d-1} b): nG rows of
  // d ints, S first (lexicographic), then beta(S) (lexicographic over gamma).
  std::vector<int> off;
};

// Assembly of one set instance's block row P(S, gamma(S)) into one front.
struct AsmBlock {
  int front;      // front index
  int type;       // set type index
  int anchor;     // leaf box index (C order over m^d)
  int rowpos;     // offset into Plan::pos of nS row positions (-1: skip)
  int colpos;     // offset into Plan::pos of nG column positions (-1: skip)
};

struct Front {
  int level = 0;
  int F = 0, p = 0;             // front order and number of pivots
  int parent = -1;
  int slot = 0;                 // index among the parent's children
  int idx = 0;                  // offset into Plan::idx (F global points, pivots first)
  int map = 0;                  // offset into Plan::map (F - p parent positions)
  int64_t off = 0;              // offset (complex elements) of the F x F front in the arena
  int64_t voff = 0;             // offset (complex elements) of the front's solve vector
  // Where the substitution reads the factor (see layout_plan): the first p
  // columns (F x p, leading dimension F) at foff, U12 (p x (F - p), leading
  // dimension ldu) at uoff, in the arena (resident storage) or in the
  // factor store (streamed storage).
  int64_t foff = 0, uoff = 0;
  int ldu = 0;
  std::vector<int> children;
};

struct Level {
  int begin = 0, end = 0;       // fronts [begin, end)
  int maxF = 0, maxP = 0;
  int maxK = 0;                 // largest F - p (fronts of a batch level differ)
  int max_children = 0;
  int blk_begin = 0, blk_end = 0;   // assembly blocks of this level
  int64_t arena_lo = 0, arena_hi = 0;   // arena range of the level's fronts
};

struct Plan {
  int d = 0, n = 0, b = 0, m = 0;
  int pattern = 0, bs = 0;      // stencil sets and their box width (see build_plan)
  int nc = 1;                   // unknowns per grid point (see expand_plan)
  int64_t N = 0;                // grid points
  int order = 0;
  std::vector<SetType> types;
  std::vector<Front> fronts;
  std::vector<Level> levels;
  std::vector<AsmBlock> blocks;
  std::vector<int> pos;         // row/column position pool for AsmBlocks
  std::vector<int> idx;         // global point indices of every front
  std::vector<int> map;         // boundary -> parent position maps
  int storage = 0;              // 0 resident, 1 streamed (see layout_plan)
  int64_t arena_elems = 0;      // front arena (complex elements, padded)
  int64_t fstore_elems = 0;     // factor store (streamed storage), else 0
  int64_t vec_elems = 0;        // sum of F (per right-hand side)
  int64_t factor_entries = 0;   // sum of p^2 + 2 p (F - p)
  double factor_flops = 0;      // real flops of all partial factorisations
  int max_front = 0;
};

// Host form of the per-front descriptor the kernels read (FrontDev), plus the
// other flat tables derived from a plan.  Every index a kernel forms from a
// front lies inside one of these ranges (tests/plan_check.cpp checks them).
struct FrontTable {
  int64_t off = 0;     // F x F front in the arena
  int64_t voff = 0;    // solve-vector slot (F positions)
  int64_t xoff = 0;    // inverse work slot (2 p F), relative to its level's base
  int64_t foff = 0, uoff = 0;   // factor read by the substitution (see Front)
  int ldu = 0;
  int F = 0, p = 0;
  int idx = 0;         // Plan::idx offset (F global points)
  int map = 0;         // Plan::map offset (F - p parent positions)
  int perm = 0;        // p permutation entries
  int dblk = 0;        // ceil(p / 32) diagonal-block inverse slots
  int inst = 0;        // problem of a batch
  int parent = -1;
  int nchild = 0;
  int child[8] = {0};
  int gptr = 0;        // F + 1 offsets into PlanTables::gsrc
};

struct PlanTables {
  std::vector<FrontTable> fronts;
  std::vector<int> gptr;            // per front F + 1 offsets into gsrc
  std::vector<int64_t> gsrc;        // vector-arena slot of each child boundary row
  std::vector<double> level_ent;    // per level: sum p(p-1)/2, p(p+1)/2, (F-p)p
  std::vector<std::vector<int>> level_F, level_p;
  int perm_total = 0;
  int dblk_total = 0;
  int64_t xwork_elems = 0;          // largest per-level inverse work
};

// Storage of the fronts (complex elements, each block padded to 16):
//  resident (0): every front F x F at its own arena offset for the whole
//    factor's life; the substitution reads the factor in place (foff = off,
//    uoff = off + p F, ldu = F).
//  streamed (1): the arena holds the fronts of two adjacent levels only, the
//    even levels from its start and the odd levels against its end, so a
//    level's fronts never overlap its children's (whose Schur complements
//    it adds) and overwrite only fronts two levels down; each front's factor
//    part (its first p columns and the U12 rows) is copied to a compact
//    factor store after the level is factored (foff, uoff = foff + p F,
//    ldu = p).  The arena is max over levels of (this level + the level
//    below) instead of the sum over all fronts.
// Also sets the solve-vector offsets and the factor counts.
void layout_plan(Plan& P, int storage);

// Builds the tables of a plan (front_inst: problem of each front).
std::string build_tables(const Plan& P, const std::vector<int>& front_inst, PlanTables& T);

// Checks d in {2,3}, n even, b | n and n / b a power of two >= 2; returns an
// empty string if valid, else a message.
std::string validate_grid(int d, int n, int b);

// Builds the plan; returns an empty string on success, else a message.
// pattern 0: stencil sets from the leaf boxes of width b (cells, faces,
// edges, vertices; Section 2.3); 1: every point its own set with the
// neighbourhood mu(j) = gamma({j}) (set boxes of width 1).  The fronts use
// leaf boxes of width b either way.
std::string build_plan(int d, int n, int b, int order, Plan& plan, int pattern = 0);

// Vector fields (nc unknowns per grid point, e.g. the d components of the
// Maxwell field): every front row of a point becomes nc rows, point-major
// (row k nc + c for the point's row k and component c), and every list that
// names points names their nc unknowns in the same order: the fronts' global
// indices (unknown (c, j) of a component-major vector of nc N entries is
// c N + j), the boundary maps and the assembly positions (set lists are
// point-major too, matching stencils computed over the sets' unknowns in
// that order).  Set types keep their point counts and offsets.  F, p and the
// level sizes grow by nc; offsets and counts are laid out again (resident).
std::string expand_plan(Plan& plan, int nc);

// Concatenates the plans of a batch of problems level by level, aligned at
// the leaves, so that one launch per level covers the fronts of every
// problem.  front_inst[f] is the problem of combined front f.  Index pools
// stay problem-local (grid indices, front positions); front, child, arena and
// vector offsets are renumbered.  All plans must have the same dimension.
std::string combine_plans(const std::vector<const Plan*>& plans, Plan& out, std::vector<int>& front_inst);

}  // namespace spp
