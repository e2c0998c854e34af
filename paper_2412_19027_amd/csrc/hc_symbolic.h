// Symbolic analysis of the Schur complement's graph (host, once per
// structure): a fill-reducing ordering, the elimination tree, the column
// counts of the Cholesky factor, fundamental supernodes and their level sets
// (the setup step of Algorithm 1; the ordering and symbolic analysis the
// linear-system layer of Sec. 3.7 relies on).
#pragma once
#include <cstdint>
#include <vector>

namespace hc {

// symmetric graph: adjacency lists without self loops or duplicates
struct SymGraph {
  int32_t n = 0;
  std::vector<int64_t> ptr;   // n + 1
  std::vector<int32_t> adj;
};

// Approximate minimum degree ordering on the quotient graph (eliminated
// vertices become elements whose variable lists stand for the cliques they
// create; elements covered by a newer one are absorbed; indistinguishable
// variables are merged into supervariables; the degree of a variable is the
// weighted size of its variable neighbours plus, per adjacent element, the
// part of that element outside the newest one, capped by the number of
// variables left).  order[k] = the vertex eliminated k-th.
// With max_work > 0 the ordering gives up (returns an empty order) once the
// element lists it has formed hold more than max_work entries in total.
std::vector<int32_t> amd_order(const SymGraph& g, int64_t max_work = 0);

// Elimination tree under `order`, in positions: parent[k] is the position of
// the parent of the k-th eliminated vertex, -1 for a root.
std::vector<int32_t> elimination_tree(const SymGraph& g, const std::vector<int32_t>& order);

// Postorder of a forest given by parent links (children before their parent,
// each subtree contiguous, roots and children in increasing label order):
// post[k] = the label placed k-th.
std::vector<int32_t> tree_postorder(const std::vector<int32_t>& parent);

// Nonzeros of each column of the Cholesky factor (diagonal included) under
// `order`, whose elimination tree is `parent` (positions).
std::vector<int64_t> column_counts(const SymGraph& g, const std::vector<int32_t>& order,
                                   const std::vector<int32_t>& parent);

// Fundamental supernodes of a postordered elimination tree: column k + 1
// joins k's supernode when it is k's parent, k is its only child and
// count[k] = count[k + 1] + 1.  Levels: 0 for a supernode without children,
// else one more than its highest child (supernodes of one level are
// independent).
struct Supernodes {
  std::vector<int32_t> first;    // first column (position) of each supernode, then n
  std::vector<int32_t> parent;   // parent supernode, -1 for a root
  std::vector<int32_t> level;
  int32_t nlevels = 0;
};
Supernodes find_supernodes(const std::vector<int32_t>& parent, const std::vector<int64_t>& count);

// The whole analysis with the tree postordered: order (vertex per position),
// parent (positions), column counts, supernodes.
struct SymbolicPlan {
  std::vector<int32_t> order, parent;
  std::vector<int64_t> count;
  Supernodes sn;
  int64_t nnz_l = 0;        // sum of the column counts
  double flops = 0;         // sum over columns of count^2 (multiply-adds of the factorisation)
};
SymbolicPlan symbolic_analysis(const SymGraph& g);

}  // namespace hc
