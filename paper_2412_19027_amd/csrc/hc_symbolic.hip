// Symbolic analysis (host code): approximate minimum degree ordering,
// elimination tree, postorder, column counts, fundamental supernodes and
// their level sets.
#include "hc_symbolic.h"

#include <algorithm>
#include <numeric>

namespace hc {

namespace {

// degree lists of the principal variables (doubly linked, one list per
// weighted degree)
struct DegreeLists {
  std::vector<int32_t> head, next, prev;
  std::vector<int64_t> at;   // list a variable is in, -1 if none
  int64_t low = 0;           // no list below this one is non-empty
  explicit DegreeLists(int32_t n) : head(n + 1, -1), next(n, -1), prev(n, -1), at(n, -1) {}
  void insert(int32_t v, int64_t d) {
    d = std::max<int64_t>(0, std::min<int64_t>(d, (int64_t)head.size() - 1));
    next[v] = head[d];
    prev[v] = -1;
    if (head[d] >= 0) prev[head[d]] = v;
    head[d] = v;
    at[v] = d;
    low = std::min(low, d);
  }
  void remove(int32_t v) {
    const int64_t d = at[v];
    if (d < 0) return;
    if (prev[v] >= 0) next[prev[v]] = next[v];
    else head[d] = next[v];
    if (next[v] >= 0) prev[next[v]] = prev[v];
    at[v] = -1;
  }
  int32_t pop_min() {
    while (low < (int64_t)head.size() && head[low] < 0) ++low;
    if (low >= (int64_t)head.size()) return -1;
    const int32_t v = head[low];
    remove(v);
    return v;
  }
};

enum VertexKind : char { VAR = 0, ELEMENT = 1, MERGED = 2, ABSORBED = 3 };

}  // namespace

std::vector<int32_t> amd_order(const SymGraph& g, int64_t max_work) {
  const int32_t n = g.n;
  std::vector<std::vector<int32_t>> A(n), E(n), L(n), members(n);
  std::vector<int64_t> nv(n, 1), deg(n, 0), w(n, 0);
  std::vector<char> kind(n, VAR);
  std::vector<int64_t> vmark(n, 0), emark(n, 0);
  int64_t vstamp = 0, estamp = 0;
  DegreeLists lists(n);
  for (int32_t i = 0; i < n; ++i) {
    members[i].push_back(i);
    for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k)
      if (g.adj[k] != i) A[i].push_back(g.adj[k]);
    std::sort(A[i].begin(), A[i].end());
    A[i].erase(std::unique(A[i].begin(), A[i].end()), A[i].end());
    deg[i] = (int64_t)A[i].size();
    lists.insert(i, deg[i]);
  }
  std::vector<int32_t> order;
  order.reserve(n);
  int64_t remaining = n;   // variables not yet eliminated (weighted)
  int64_t work = 0;        // entries of the element lists formed so far
  std::vector<int32_t> Lp;
  std::vector<std::pair<int64_t, int32_t>> hashed;
  while ((int32_t)order.size() < n) {
    const int32_t p = lists.pop_min();
    if (p < 0) break;   // cannot happen while variables remain
    // the new element's variables: p's variable neighbours and the members of
    // its adjacent elements, which p's elimination covers (they are absorbed)
    ++vstamp;
    vmark[p] = vstamp;
    Lp.clear();
    auto add = [&](int32_t v) {
      if (kind[v] == VAR && nv[v] > 0 && vmark[v] != vstamp) {
        vmark[v] = vstamp;
        Lp.push_back(v);
      }
    };
    for (int32_t v : A[p]) add(v);
    for (int32_t e : E[p])
      if (kind[e] == ELEMENT) {
        for (int32_t v : L[e]) add(v);
        kind[e] = ABSORBED;
        std::vector<int32_t>().swap(L[e]);
      }
    kind[p] = ELEMENT;
    std::vector<int32_t>().swap(A[p]);
    std::vector<int32_t>().swap(E[p]);
    for (int32_t v : members[p]) order.push_back(v);
    std::vector<int32_t>().swap(members[p]);
    remaining -= nv[p];
    int64_t lp_weight = 0;
    for (int32_t v : Lp) {
      lp_weight += nv[v];
      lists.remove(v);
    }
    L[p] = Lp;
    work += (int64_t)Lp.size();
    if (max_work > 0 && work > max_work) return {};
    // element lists gain p and lose absorbed elements; variable lists lose what p covers
    for (int32_t v : Lp) {
      auto& ev = E[v];
      ev.erase(std::remove_if(ev.begin(), ev.end(), [&](int32_t e) { return kind[e] != ELEMENT; }), ev.end());
      ev.push_back(p);
      auto& av = A[v];
      av.erase(std::remove_if(av.begin(), av.end(),
                              [&](int32_t u) { return kind[u] != VAR || nv[u] == 0 || vmark[u] == vstamp; }),
               av.end());
    }
    // w(e) = weighted |L_e \ L_p| for the other elements adjacent to L_p
    ++estamp;
    for (int32_t v : Lp)
      for (int32_t e : E[v]) {
        if (e == p) continue;
        if (emark[e] != estamp) {
          emark[e] = estamp;
          auto& le = L[e];
          le.erase(std::remove_if(le.begin(), le.end(), [&](int32_t u) { return kind[u] != VAR || nv[u] == 0; }),
                   le.end());
          int64_t s = 0;
          for (int32_t u : le) s += nv[u];
          w[e] = s;
        }
        w[e] -= nv[v];
      }
    // elements inside L_p are absorbed; approximate external degrees
    for (int32_t v : Lp) {
      auto& ev = E[v];
      int64_t d = lp_weight - nv[v];
      ev.erase(std::remove_if(ev.begin(), ev.end(),
                              [&](int32_t e) {
                                if (e == p) return false;
                                if (w[e] <= 0) {   // L_e is inside L_p: absorbed into p
                                  kind[e] = ABSORBED;
                                  return true;
                                }
                                return false;
                              }),
               ev.end());
      for (int32_t e : ev)
        if (e != p) d += w[e];
      for (int32_t u : A[v]) d += nv[u];
      deg[v] = std::min<int64_t>(d, remaining - nv[v]);
    }
    // supervariables: variables of L_p with the same element and variable
    // neighbours are merged
    hashed.clear();
    for (int32_t v : Lp) {
      std::sort(E[v].begin(), E[v].end());
      std::sort(A[v].begin(), A[v].end());
      int64_t h = 0;
      for (int32_t e : E[v]) h += e;
      for (int32_t u : A[v]) h += u;
      hashed.emplace_back(h * 1000003 + (int64_t)(E[v].size() + 31 * A[v].size()), v);
    }
    std::sort(hashed.begin(), hashed.end());
    for (size_t a = 0; a < hashed.size();) {
      size_t b = a;
      while (b < hashed.size() && hashed[b].first == hashed[a].first) ++b;
      for (size_t x = a; x < b; ++x) {
        const int32_t v = hashed[x].second;
        if (nv[v] == 0) continue;
        for (size_t y = x + 1; y < b; ++y) {
          const int32_t u = hashed[y].second;
          if (nv[u] == 0 || E[u] != E[v] || A[u] != A[v]) continue;
          nv[v] += nv[u];
          deg[v] -= nv[u];
          nv[u] = 0;
          kind[u] = MERGED;
          members[v].insert(members[v].end(), members[u].begin(), members[u].end());
          std::vector<int32_t>().swap(members[u]);
          std::vector<int32_t>().swap(A[u]);
          std::vector<int32_t>().swap(E[u]);
        }
      }
      a = b;
    }
    for (int32_t v : Lp)
      if (kind[v] == VAR && nv[v] > 0) lists.insert(v, std::max<int64_t>(0, deg[v]));
  }
  return order;
}

std::vector<int32_t> elimination_tree(const SymGraph& g, const std::vector<int32_t>& order) {
  const int32_t n = g.n;
  std::vector<int32_t> pos(n), parent(n, -1), anc(n, -1);
  for (int32_t k = 0; k < n; ++k) pos[order[k]] = k;
  // for each column k, each earlier neighbour's current root (found by
  // walking ancestor links, which are compressed to k on the way) becomes a
  // child of k
  for (int32_t k = 0; k < n; ++k) {
    const int32_t v = order[k];
    for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
      int32_t i = pos[g.adj[e]];
      while (i != -1 && i < k) {
        const int32_t up = anc[i];
        anc[i] = k;
        if (up == -1) parent[i] = k;
        i = up;
      }
    }
  }
  return parent;
}

std::vector<int32_t> tree_postorder(const std::vector<int32_t>& parent) {
  const int32_t n = (int32_t)parent.size();
  std::vector<int32_t> head(n, -1), nxt(n, -1), post;
  post.reserve(n);
  for (int32_t j = n - 1; j >= 0; --j)   // children lists in increasing order
    if (parent[j] >= 0) {
      nxt[j] = head[parent[j]];
      head[parent[j]] = j;
    }
  std::vector<int32_t> stack;
  for (int32_t r = 0; r < n; ++r) {
    if (parent[r] != -1) continue;
    stack.push_back(r);
    while (!stack.empty()) {
      const int32_t v = stack.back();
      if (head[v] >= 0) {   // descend into the next unvisited child
        const int32_t c = head[v];
        head[v] = nxt[c];
        stack.push_back(c);
      } else {
        stack.pop_back();
        post.push_back(v);
      }
    }
  }
  return post;
}

std::vector<int64_t> column_counts(const SymGraph& g, const std::vector<int32_t>& order,
                                   const std::vector<int32_t>& parent) {
  // row structure of each column: its later neighbours plus its children's
  // structures (without the column itself); children are merged into the
  // parent and then released
  const int32_t n = g.n;
  std::vector<int32_t> pos(n);
  for (int32_t k = 0; k < n; ++k) pos[order[k]] = k;
  std::vector<std::vector<int32_t>> kids(n), st(n);
  for (int32_t k = 0; k < n; ++k)
    if (parent[k] >= 0) kids[parent[k]].push_back(k);
  std::vector<int32_t> mark(n, -1);
  std::vector<int64_t> count(n, 1);
  for (int32_t k = 0; k < n; ++k) {
    auto& s = st[k];
    mark[k] = k;
    const int32_t v = order[k];
    for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
      const int32_t i = pos[g.adj[e]];
      if (i > k && mark[i] != k) {
        mark[i] = k;
        s.push_back(i);
      }
    }
    for (int32_t c : kids[k]) {
      for (int32_t i : st[c])
        if (i > k && mark[i] != k) {
          mark[i] = k;
          s.push_back(i);
        }
      std::vector<int32_t>().swap(st[c]);
    }
    count[k] = 1 + (int64_t)s.size();
  }
  return count;
}

Supernodes find_supernodes(const std::vector<int32_t>& parent, const std::vector<int64_t>& count) {
  const int32_t n = (int32_t)parent.size();
  std::vector<int32_t> nkids(n, 0);
  for (int32_t k = 0; k < n; ++k)
    if (parent[k] >= 0) nkids[parent[k]]++;
  Supernodes s;
  std::vector<int32_t> sn_of(n);
  for (int32_t k = 0; k < n; ++k) {
    const bool join = k > 0 && parent[k - 1] == k && nkids[k] == 1 && count[k - 1] == count[k] + 1;
    if (!join) s.first.push_back(k);
    sn_of[k] = (int32_t)s.first.size() - 1;
  }
  const int32_t ns = (int32_t)s.first.size();
  s.first.push_back(n);
  s.parent.assign(ns, -1);
  for (int32_t t = 0; t < ns; ++t) {
    const int32_t last = s.first[t + 1] - 1;
    if (parent[last] >= 0) s.parent[t] = sn_of[parent[last]];
  }
  // postordered tree: children come before their parent
  s.level.assign(ns, 0);
  for (int32_t t = 0; t < ns; ++t)
    if (s.parent[t] >= 0) s.level[s.parent[t]] = std::max(s.level[s.parent[t]], s.level[t] + 1);
  s.nlevels = ns ? 1 + *std::max_element(s.level.begin(), s.level.end()) : 0;
  return s;
}

SymbolicPlan symbolic_analysis(const SymGraph& g) {
  SymbolicPlan P;
  const std::vector<int32_t> o = amd_order(g);
  const std::vector<int32_t> par = elimination_tree(g, o);
  const std::vector<int32_t> post = tree_postorder(par);
  P.order.resize(g.n);
  for (int32_t k = 0; k < g.n; ++k) P.order[k] = o[post[k]];   // same tree, children first
  P.parent = elimination_tree(g, P.order);
  P.count = column_counts(g, P.order, P.parent);
  P.sn = find_supernodes(P.parent, P.count);
  for (int64_t c : P.count) {
    P.nnz_l += c;
    P.flops += (double)c * (double)c;
  }
  return P;
}

}  // namespace hc
