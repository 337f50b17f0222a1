// Contraction order (greedy pairwise, randomised restarts) and slice choice.
//
// The paper refers its order search to earlier work that is not reproduced
// here; this is a plain greedy: repeatedly merge the pair of tensors sharing
// an index whose merge changes the total stored size the least
// (size(C) - size(A) - size(B)), with Gumbel-perturbed scores on restarts.
// Slicing (the paper's preprocessing into equal-cost subtasks) then fixes, one
// at a time, the index whose removal most reduces the largest intermediate
// and, as a tie-break, the flops of one slice.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <queue>
#include <thread>

#include "plan.h"

namespace qc {

namespace {

// SplitMix64 (Steele, Lea and Flood 2014).
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
    double gumbel() {
        double u = uniform();
        u = std::min(std::max(u, 1e-300), 1.0 - 1e-16);
        return -std::log(-std::log(u));
    }
};

std::vector<int> sorted_union(const std::vector<int> &a, const std::vector<int> &b) {
    std::vector<int> out;
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
    return out;
}

}  // namespace

std::vector<Merge> greedy_order(const OrderProblem &p, const std::vector<char> &removed,
                                uint64_t seed, double temperature) {
    return greedy_order_phased(p, removed, seed, temperature, nullptr, 0);
}

// With `dynamic` set: a first phase merges only pairs of tensors that are both
// free of dynamic leaves (sliced or output indices) while the result keeps at
// most `const_cap` indices, so that the pair-invariant part of the network
// ends up in subtrees of its own; then the plain greedy finishes.
std::vector<Merge> greedy_order_phased(const OrderProblem &p, const std::vector<char> &removed, uint64_t seed,
                                       double temperature, const std::vector<char> *dynamic, int const_cap) {
    const int L = (int)p.leaf_idx.size();
    std::vector<std::vector<int>> sets;
    sets.reserve(2 * L);
    std::vector<std::vector<int>> holders(p.n_index);
    for (int t = 0; t < L; ++t) {
        std::vector<int> s;
        for (int e : p.leaf_idx[t])
            if (!removed[e]) s.push_back(e);
        std::sort(s.begin(), s.end());
        for (int e : s) holders[e].push_back(t);
        sets.push_back(std::move(s));
    }
    std::vector<char> alive(L, 1);
    Rng rng{seed};
    struct Cand { double key; int a, b; };
    auto cmp = [](const Cand &x, const Cand &y) {
        if (x.key != y.key) return x.key > y.key;
        if (x.a != y.a) return x.a > y.a;
        return x.b > y.b;
    };
    std::priority_queue<Cand, std::vector<Cand>, decltype(cmp)> heap(cmp);
    auto result_rank = [&](int a, int b) {
        int r = 0;
        const auto &A = sets[a], &B = sets[b];
        size_t i = 0, j = 0;
        while (i < A.size() || j < B.size()) {
            if (j == B.size() || (i < A.size() && A[i] < B[j])) { ++r; ++i; }
            else if (i == A.size() || B[j] < A[i]) { ++r; ++j; }
            else {  // shared: stays if another live tensor holds it (or it is never summed)
                if (holders[A[i]].size() > 2 || p.kept(A[i])) ++r;
                ++i; ++j;
            }
        }
        return r;
    };
    std::vector<char> is_dyn(L, 0);
    if (dynamic)
        for (int t = 0; t < L; ++t) is_dyn[t] = (*dynamic)[t];
    bool phase1 = dynamic != nullptr;
    auto push = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        const int rc = result_rank(a, b);
        if (phase1 && (is_dyn[a] || is_dyn[b] || rc > const_cap)) return;
        const double sa = std::ldexp(1.0, (int)sets[a].size()), sb = std::ldexp(1.0, (int)sets[b].size());
        double key = std::ldexp(1.0, rc) - sa - sb;
        if (temperature > 0) key -= temperature * (sa + sb) * rng.gumbel();
        heap.push(Cand{key, a, b});
    };
    auto push_all = [&]() {
        for (int e = 0; e < p.n_index; ++e)
            for (size_t i = 0; i < holders[e].size(); ++i)
                for (size_t j = i + 1; j < holders[e].size(); ++j) push(holders[e][i], holders[e][j]);
    };
    push_all();

    std::vector<Merge> tree;
    int n_alive = L;
    auto do_merge = [&](int a, int b) {
        std::vector<int> c;
        const std::vector<int> u = sorted_union(sets[a], sets[b]);
        for (int e : u) {
            const bool both = std::binary_search(sets[a].begin(), sets[a].end(), e) &&
                              std::binary_search(sets[b].begin(), sets[b].end(), e);
            if (!(both && holders[e].size() == 2 && !p.kept(e))) c.push_back(e);
        }
        const int id = (int)sets.size();
        for (int e : u) {
            auto &h = holders[e];
            h.erase(std::remove_if(h.begin(), h.end(), [&](int t) { return t == a || t == b; }), h.end());
        }
        for (int e : c) holders[e].push_back(id);
        sets.push_back(std::move(c));
        alive[a] = alive[b] = 0;
        alive.push_back(1);
        is_dyn.push_back(is_dyn[a] || is_dyn[b]);
        tree.push_back(Merge{a, b});
        --n_alive;
        return id;
    };
    for (;;) {
        while (!heap.empty()) {
            Cand cd = heap.top();
            heap.pop();
            if (!alive[cd.a] || !alive[cd.b]) continue;
            const int id = do_merge(cd.a, cd.b);
            std::vector<int> nbr;
            for (int e : sets[id])
                for (int d : holders[e])
                    if (d != id) nbr.push_back(d);
            std::sort(nbr.begin(), nbr.end());
            nbr.erase(std::unique(nbr.begin(), nbr.end()), nbr.end());
            for (int d : nbr) push(id, d);
        }
        if (!phase1) break;
        phase1 = false;
        push_all();
    }
    // Disconnected pieces: fold the two smallest until one tensor is left.
    while (n_alive > 1) {
        int a = -1, b = -1;
        for (int t = 0; t < (int)sets.size(); ++t) {
            if (!alive[t]) continue;
            if (a < 0 || sets[t].size() < sets[a].size()) { b = a; a = t; }
            else if (b < 0 || sets[t].size() < sets[b].size()) b = t;
        }
        do_merge(std::min(a, b), std::max(a, b));
    }
    return tree;
}

// Per-node index sets with indices closed once all leaves holding them have
// been merged.
static void node_sets(const OrderProblem &p, const std::vector<Merge> &tree,
                      const std::vector<char> &removed, std::vector<std::vector<int>> &sets,
                      std::vector<std::vector<int>> &unions) {
    const int L = (int)p.leaf_idx.size();
    std::vector<int> total(p.n_index, 0);
    std::vector<std::vector<std::pair<int, int>>> cnt;
    sets.clear();
    unions.assign(tree.size(), {});
    for (int t = 0; t < L; ++t) {
        std::vector<int> s;
        for (int e : p.leaf_idx[t])
            if (!removed[e]) { s.push_back(e); ++total[e]; }
        std::sort(s.begin(), s.end());
        std::vector<std::pair<int, int>> c;
        for (int e : s) c.push_back({e, 1});
        cnt.push_back(std::move(c));
        sets.push_back(std::move(s));
    }
    for (int e = 0; e < p.n_index; ++e) total[e] += p.kept(e);  // open outputs are never closed
    for (size_t i = 0; i < tree.size(); ++i) {
        const auto &ca = cnt[tree[i].a], &cb = cnt[tree[i].b];
        std::vector<std::pair<int, int>> cc;
        std::vector<int> s, u;
        size_t x = 0, y = 0;
        while (x < ca.size() || y < cb.size()) {
            std::pair<int, int> v;
            if (y == cb.size() || (x < ca.size() && ca[x].first < cb[y].first)) v = ca[x++];
            else if (x == ca.size() || cb[y].first < ca[x].first) v = cb[y++];
            else { v = {ca[x].first, ca[x].second + cb[y].second}; ++x; ++y; }
            u.push_back(v.first);
            if (v.second < total[v.first]) { cc.push_back(v); s.push_back(v.first); }
        }
        cnt.push_back(std::move(cc));
        sets.push_back(std::move(s));
        unions[i] = std::move(u);
    }
}

TreeCost tree_cost(const OrderProblem &p, const std::vector<Merge> &tree,
                   const std::vector<char> &removed) {
    std::vector<std::vector<int>> sets, unions;
    node_sets(p, tree, removed, sets, unions);
    TreeCost c;
    const int L = (int)p.leaf_idx.size();
    double live = 0;
    for (int t = 0; t < L; ++t) {
        c.max_log2 = std::max(c.max_log2, (double)sets[t].size());
        live += 8.0 * std::ldexp(1.0, (int)sets[t].size());
    }
    c.peak_live = live;
    for (size_t i = 0; i < tree.size(); ++i) {
        const double sa = std::ldexp(1.0, (int)sets[tree[i].a].size());
        const double sb = std::ldexp(1.0, (int)sets[tree[i].b].size());
        const double sc = std::ldexp(1.0, (int)sets[L + i].size());
        c.max_log2 = std::max(c.max_log2, (double)sets[L + i].size());
        c.flops += 8.0 * std::ldexp(1.0, (int)unions[i].size());
        c.bytes += 8.0 * (sa + sb + sc);
        live += 8.0 * sc;
        c.peak_live = std::max(c.peak_live, live);
        live -= 8.0 * (sa + sb);
    }
    return c;
}

// Chooses sliced indices on a fixed tree.  Returns false if the cap cannot be
// met.  `sliced` may hold explicit choices on entry.
static bool choose_slices(const OrderProblem &p, const std::vector<Merge> &tree, int k_target,
                          double cap_log2, std::vector<int> &sliced, const std::vector<char> &sliceable,
                          double &achieved_log2, int max_add = 1 << 30) {
    std::vector<char> removed(p.n_index, 0);
    for (int e : sliced) removed[e] = 1;
    for (int added = 0;; ++added) {
        std::vector<std::vector<int>> sets, unions;
        node_sets(p, tree, removed, sets, unions);
        int maxr = 0;
        for (auto &s : sets) maxr = std::max(maxr, (int)s.size());
        achieved_log2 = maxr;
        const bool cap_ok = cap_log2 <= 0 || maxr <= cap_log2;
        if (cap_ok && (int)sliced.size() >= k_target) return true;
        if (added == max_add) return false;
        // While the cap is not met, candidates are the indices of the largest
        // nodes and the one leaving the smallest largest node wins (then the
        // fewest flops per slice); once it is met, more slices are wanted only
        // for k, and any sliceable index may be taken: the one leaving the
        // fewest flops per slice (the least total work over all slices).
        std::vector<char> cand(p.n_index, 0);
        if (cap_ok) {
            for (int e = 0; e < p.n_index; ++e) cand[e] = sliceable[e] && !removed[e];
        } else {
            for (auto &s : sets)
                if ((int)s.size() == maxr)
                    for (int e : s) cand[e] = sliceable[e] && !removed[e];
        }
        int best = -1;
        int best_max = 1 << 30;
        double best_flops = 0;
        for (int e = 0; e < p.n_index; ++e) {
            if (!cand[e]) continue;
            int m = 0;
            if (!cap_ok)
                for (auto &s : sets) m = std::max(m, (int)s.size() - (int)std::binary_search(s.begin(), s.end(), e));
            double f = 0;
            for (auto &u : unions)
                f += std::ldexp(1.0, (int)u.size() - (int)std::binary_search(u.begin(), u.end(), e));
            if (best < 0 || m < best_max || (m == best_max && f < best_flops)) {
                best = e; best_max = m; best_flops = f;
            }
        }
        if (best < 0) return cap_ok && (int)sliced.size() >= k_target;  // nothing left to slice
        removed[best] = 1;
        sliced.push_back(best);
    }
}

// Largest pair-invariant intermediate folded on the host (log2 entries).
constexpr int kFoldMaxLog2 = 14;

// Per-(slice, bitstring) flops of a tree once its foldable pair-invariant
// subtrees are precomputed.
// Estimated device cost of one pairwise step, in complex multiply-adds: the
// larger of its multiply-adds and w times the elements it reads and writes
// (w = 20: a roofline with ~100 TFLOP/s of complex FP32 arithmetic against
// ~5 TB/s of memory traffic), so that steps moving large tensors for little
// arithmetic are charged for their traffic.
constexpr double kMovePerMac = 20.0;
// The full search also runs under this weight and keeps whichever result is
// cheaper under kMovePerMac: the randomised search settles in different trees
// under different weights, and on the 70-qubit workload the tree found under
// this one is cheaper under both (half the flops and bytes per slice).
constexpr double kMovePerMacAlt = 10.0;
inline double step_cost(int union_bits, int a_bits, int b_bits, int c_bits, double w) {
    const double macs = std::ldexp(1.0, union_bits);
    const double moved = std::ldexp(1.0, a_bits) + std::ldexp(1.0, b_bits) + std::ldexp(1.0, c_bits);
    return std::max(macs, w * moved);
}

// Per-(slice, bitstring) device cost of a tree once its foldable
// pair-invariant subtrees are precomputed: the objective of the search.
static double per_pair_cost(const OrderProblem &p, const std::vector<Merge> &tree,
                             const std::vector<char> &removed, const std::vector<char> &dyn_leaf) {
    std::vector<std::vector<int>> sets, unions;
    node_sets(p, tree, removed, sets, unions);
    const int L = (int)p.leaf_idx.size();
    std::vector<char> dyn(dyn_leaf.begin(), dyn_leaf.end());
    double f = 0;
    for (size_t i = 0; i < tree.size(); ++i) {
        const bool d = dyn[tree[i].a] || dyn[tree[i].b];
        dyn.push_back(d);
        if (d || (int)sets[L + i].size() > kFoldMaxLog2)
            f += step_cost((int)unions[i].size(), (int)sets[tree[i].a].size(), (int)sets[tree[i].b].size(),
                           (int)sets[L + i].size(), p.move_per_mac);
    }
    return f;
}

// ------------------------------------------------- subtree reconfiguration
// Improves a tree locally: for a node r, its subtree is cut at a frontier F of
// up to kReconfFrontier nodes (grown from r's children by opening the most
// expensive internal frontier node first), and the order in which F's tensors
// are contracted into r is replaced by the cheapest one, found by dynamic
// programming over the subsets of F.  An index is open at a subset S of F
// when some leaf under S holds it and some leaf outside S does, so every
// subset has a fixed index set and the cost of a merge A + B is 2^|open(A)
// U open(B)|.  Merges of tensors free of dynamic leaves that stay within the
// host-folding limits cost nothing (they are evaluated once on the host).
// A new tree is kept only if its per-(slice, bitstring) work -- the objective
// of the search -- goes down and no intermediate exceeds the cap.
constexpr int kReconfFrontier = 10;
constexpr int kReconfMaxIdx = 128;
constexpr int kReconfSweeps = 6;

namespace {

struct TreeShape {
    int L = 0;
    std::vector<int> a, b;        // children of node L + i
    int root = -1;
};

TreeShape shape_of(int L, const std::vector<Merge> &tree) {
    TreeShape t;
    t.L = L;
    for (const Merge &m : tree) { t.a.push_back(m.a); t.b.push_back(m.b); }
    t.root = tree.empty() ? 0 : L + (int)tree.size() - 1;
    return t;
}

// The merges of a shape in post-order from its root (children before parents).
std::vector<Merge> merges_of(const TreeShape &t) {
    std::vector<Merge> out;
    std::vector<int> id(t.L + t.a.size(), -1);
    for (int l = 0; l < t.L; ++l) id[l] = l;
    std::vector<std::pair<int, int>> st{{t.root, 0}};
    while (!st.empty()) {
        auto &[n, state] = st.back();
        if (n < t.L) { st.pop_back(); continue; }
        const int i = n - t.L;
        if (state == 0) { state = 1; st.push_back({t.a[i], 0}); continue; }
        if (state == 1) { state = 2; st.push_back({t.b[i], 0}); continue; }
        out.push_back(Merge{id[t.a[i]], id[t.b[i]]});
        id[n] = t.L + (int)out.size() - 1;
        st.pop_back();
    }
    return out;
}

struct Bits {
    uint64_t w[2] = {0, 0};
    void set(int i) { w[i >> 6] |= uint64_t(1) << (i & 63); }
    int count() const { return __builtin_popcountll(w[0]) + __builtin_popcountll(w[1]); }
    Bits operator|(const Bits &o) const { Bits r; r.w[0] = w[0] | o.w[0]; r.w[1] = w[1] | o.w[1]; return r; }
};

}  // namespace

// Open index sets and merge unions of every node of a shape (node ids as in
// the shape: leaves, then L + i for the node whose children are a[i], b[i]).
static void shape_sets(const OrderProblem &p, const TreeShape &t, const std::vector<char> &removed,
                       const std::vector<int> &total, std::vector<std::vector<int>> &sets,
                       std::vector<std::vector<int>> &unions) {
    const int N = t.L + (int)t.a.size();
    std::vector<std::vector<std::pair<int, int>>> cnt(N);
    sets.assign(N, {});
    unions.assign(N, {});
    for (int l = 0; l < t.L; ++l) {
        for (int e : p.leaf_idx[l])
            if (!removed[e]) cnt[l].push_back({e, 1});
        std::sort(cnt[l].begin(), cnt[l].end());
        for (auto &v : cnt[l]) sets[l].push_back(v.first);
    }
    std::vector<std::pair<int, int>> st{{t.root, 0}};
    while (!st.empty()) {
        auto &[n, state] = st.back();
        if (n < t.L) { st.pop_back(); continue; }
        const int i = n - t.L;
        if (state == 0) { state = 1; st.push_back({t.a[i], 0}); continue; }
        if (state == 1) { state = 2; st.push_back({t.b[i], 0}); continue; }
        const auto &ca = cnt[t.a[i]], &cb = cnt[t.b[i]];
        size_t x = 0, y = 0;
        while (x < ca.size() || y < cb.size()) {
            std::pair<int, int> v;
            if (y == cb.size() || (x < ca.size() && ca[x].first < cb[y].first)) v = ca[x++];
            else if (x == ca.size() || cb[y].first < ca[x].first) v = cb[y++];
            else { v = {ca[x].first, ca[x].second + cb[y].second}; ++x; ++y; }
            unions[n].push_back(v.first);
            if (v.second < total[v.first]) { cnt[n].push_back(v); sets[n].push_back(v.first); }
        }
        st.pop_back();
    }
}

static double reconfigure(const OrderProblem &p, std::vector<Merge> &tree, const std::vector<char> &removed,
                          const std::vector<char> &dyn_leaf, double cap, uint64_t seed, int sweeps) {
    const int L = (int)p.leaf_idx.size();
    if (tree.size() < 2) return per_pair_cost(p, tree, removed, dyn_leaf);
    std::vector<int> total(p.n_index, 0);
    for (int t = 0; t < L; ++t)
        for (int e : p.leaf_idx[t])
            if (!removed[e]) ++total[e];
    for (int e = 0; e < p.n_index; ++e) total[e] += p.kept(e);
    double best = per_pair_cost(p, tree, removed, dyn_leaf);
    Rng rng{seed};
    TreeShape t = shape_of(L, tree);
    const int N = L + (int)t.a.size();
    std::vector<std::vector<int>> sets, unions;
    std::vector<char> dyn(N, 0);
    auto refresh = [&]() {
        shape_sets(p, t, removed, total, sets, unions);
        for (int l = 0; l < L; ++l) dyn[l] = dyn_leaf[l];
        // dyn of internal nodes, children first (post-order of the shape).
        std::vector<std::pair<int, int>> st{{t.root, 0}};
        while (!st.empty()) {
            auto &[n, state] = st.back();
            if (n < L) { st.pop_back(); continue; }
            const int i = n - L;
            if (state == 0) { state = 1; st.push_back({t.a[i], 0}); continue; }
            if (state == 1) { state = 2; st.push_back({t.b[i], 0}); continue; }
            dyn[n] = dyn[t.a[i]] || dyn[t.b[i]];
            st.pop_back();
        }
    };
    refresh();
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        bool improved = false;
        // Visit internal nodes from the most expensive merge down (ties random).
        std::vector<std::pair<double, int>> order;
        for (int n = L; n < N; ++n) order.push_back({-(double)unions[n].size() - 0.5 * rng.uniform(), n});
        std::sort(order.begin(), order.end());
        for (auto &oi : order) {
            const int r = oi.second;
            // Frontier: open the most expensive internal node first.
            std::vector<int> F{t.a[r - L], t.b[r - L]};
            std::vector<int> inner{r};
            while ((int)F.size() < kReconfFrontier) {
                int pick = -1;
                for (int j = 0; j < (int)F.size(); ++j)
                    if (F[j] >= L && (pick < 0 || unions[F[j]].size() > unions[F[pick]].size())) pick = j;
                if (pick < 0) break;
                const int n = F[pick];
                inner.push_back(n);
                F[pick] = t.a[n - L];
                F.push_back(t.b[n - L]);
            }
            const int f = (int)F.size();
            if (f < 3) continue;
            // Index universe of the frontier and per-frontier leaf counts.
            std::vector<int> E;
            for (int x : F) E.insert(E.end(), sets[x].begin(), sets[x].end());
            std::sort(E.begin(), E.end());
            E.erase(std::unique(E.begin(), E.end()), E.end());
            if ((int)E.size() > kReconfMaxIdx) continue;
            std::vector<std::vector<int>> cnt(f, std::vector<int>(E.size(), 0));
            for (int x = 0; x < f; ++x) {
                std::vector<int> st{F[x]};
                while (!st.empty()) {
                    const int n = st.back();
                    st.pop_back();
                    if (n >= L) { st.push_back(t.a[n - L]); st.push_back(t.b[n - L]); continue; }
                    for (int e : p.leaf_idx[n]) {
                        if (removed[e]) continue;
                        auto it = std::lower_bound(E.begin(), E.end(), e);
                        if (it != E.end() && *it == e) ++cnt[x][it - E.begin()];
                    }
                }
            }
            const int S_all = (1 << f) - 1;
            std::vector<Bits> open(S_all + 1);
            std::vector<char> cst(S_all + 1, 1);
            std::vector<int> c(E.size());
            for (int S = 1; S <= S_all; ++S) {
                std::fill(c.begin(), c.end(), 0);
                bool cs = true;
                for (int x = 0; x < f; ++x)
                    if ((S >> x) & 1) {
                        cs = cs && !dyn[F[x]];
                        for (size_t j = 0; j < E.size(); ++j) c[j] += cnt[x][j];
                    }
                Bits bm;
                for (size_t j = 0; j < E.size(); ++j)
                    if (c[j] > 0 && c[j] < total[E[j]]) bm.set((int)j);
                open[S] = bm;
                cst[S] = cs;
            }
            const double INF = 1e300;
            std::vector<double> cost(S_all + 1, INF);
            std::vector<int> split(S_all + 1, 0);
            for (int x = 0; x < f; ++x) cost[1 << x] = 0;
            for (int S = 1; S <= S_all; ++S) {
                if (__builtin_popcount(S) < 2) continue;
                const int sz = open[S].count();
                if (cap > 0 && sz > cap) continue;
                const int low = S & -S;
                // A holds the lowest member of S; B = S \ A is nonempty.
                for (int A = (S - 1) & S; A > 0; A = (A - 1) & S) {
                    if (!(A & low)) continue;
                    const int B = S ^ A;
                    if (cost[A] >= INF || cost[B] >= INF) continue;
                    const int u = (open[A] | open[B]).count();
                    const bool folds = cst[S] && sz <= kFoldMaxLog2 && u <= kFoldMaxLog2 + 4;
                    const double v = cost[A] + cost[B] +
                                     (folds ? 0.0 : step_cost(u, open[A].count(), open[B].count(), sz, p.move_per_mac));
                    if (v < cost[S]) { cost[S] = v; split[S] = A; }
                }
            }
            if (cost[S_all] >= INF) continue;
            // Current cost of the subtree's merges under the same rule.
            double cur = 0;
            for (int n : inner) {
                const bool folds = !dyn[n] && (int)sets[n].size() <= kFoldMaxLog2 &&
                                   (int)unions[n].size() <= kFoldMaxLog2 + 4;
                cur += folds ? 0.0 : step_cost((int)unions[n].size(), (int)sets[t.a[n - L]].size(),
                                               (int)sets[t.b[n - L]].size(), (int)sets[n].size(), p.move_per_mac);
            }
            if (cost[S_all] >= cur * (1 - 1e-9)) continue;
            // Rebuild the subtree reusing the inner nodes' ids (r keeps its id).
            TreeShape t2 = t;
            std::vector<int> free_ids(inner.begin() + 1, inner.end());
            std::function<int(int, bool)> build = [&](int S, bool is_root) -> int {
                if (__builtin_popcount(S) == 1) return F[__builtin_ctz(S)];
                const int A = split[S], B = S ^ A;
                const int na = build(A, false), nb = build(B, false);
                const int id = is_root ? r : free_ids.back();
                if (!is_root) free_ids.pop_back();
                t2.a[id - L] = na;
                t2.b[id - L] = nb;
                return id;
            };
            build(S_all, true);
            std::vector<Merge> cand = merges_of(t2);
            const TreeCost tc = tree_cost(p, cand, removed);
            if (cap > 0 && tc.max_log2 > cap) continue;
            const double v = per_pair_cost(p, cand, removed, dyn_leaf);
            if (v < best * (1 - 1e-12)) {
                best = v;
                t = std::move(t2);
                tree = std::move(cand);
                refresh();
                improved = true;
            }
        }
        if (!improved) break;
    }
    return best;
}

// Replaces every maximal pair-invariant subtree (no dynamic leaf, result of
// at most 2^kFoldMaxLog2 entries) by one leaf computed here in FP64 -- the
// paper's preprocessing, done once per circuit for all slices and bitstrings.
static void fold_invariant_subtrees(qc_plan *plan, const std::vector<char> &dyn_leaf) {
    OrderProblem &p = plan->prob;
    const int L = (int)p.leaf_idx.size();
    const int M = (int)plan->tree.size();
    std::vector<char> removed(p.n_index, 0);
    for (int e : plan->sliced) removed[e] = 1;
    std::vector<std::vector<int>> sets, unions;
    node_sets(p, plan->tree, removed, sets, unions);
    std::vector<char> foldable(L + M, 0), cst(L + M, 0);
    for (int t = 0; t < L; ++t) cst[t] = !dyn_leaf[t];
    std::vector<int> parent(L + M, -1);
    for (int i = 0; i < M; ++i) {
        const int n = L + i;
        const int a = plan->tree[i].a, b = plan->tree[i].b;
        cst[n] = cst[a] && cst[b];
        // Every node of a folded subtree must be small, so the host work stays
        // bounded (2^|union| products per step).
        foldable[n] = cst[n] && (int)sets[n].size() <= kFoldMaxLog2 && (int)unions[i].size() <= kFoldMaxLog2 + 4 &&
                      (a < L || foldable[a]) && (b < L || foldable[b]);
        parent[plan->tree[i].a] = parent[plan->tree[i].b] = n;
    }
    std::vector<char> top(L + M, 0), inside(L + M, 0);
    for (int n = L + M - 1; n >= L; --n) {
        if (!foldable[n]) continue;
        if (parent[n] >= 0 && (foldable[parent[n]] || inside[parent[n]])) inside[n] = 1;
        else top[n] = 1;
    }
    // Children of folded nodes are inside as well.
    for (int n = L + M - 1; n >= L; --n)
        if (top[n] || inside[n]) inside[plan->tree[n - L].a] = inside[plan->tree[n - L].b] = 1;
    bool any = false;
    for (int n = L; n < L + M; ++n) any |= top[n];
    if (!any) return;
    // Host values of the folded nodes (post-order).
    double folded_flops = 0;
    std::vector<Tensor> val(L + M);
    std::vector<char> have(L + M, 0);
    for (int t = 0; t < L; ++t)
        if (inside[t]) { val[t] = plan->net.leaves[t]; have[t] = 1; }
    for (int i = 0; i < M; ++i) {
        const int n = L + i;
        if (!(inside[n] || top[n])) continue;
        const int a = plan->tree[i].a, b = plan->tree[i].b;
        std::vector<int> contracted;
        for (int e : unions[i])
            if (!std::binary_search(sets[n].begin(), sets[n].end(), e)) contracted.push_back(e);
        val[n] = contract_host(val[a], val[b], sets[n], contracted);
        folded_flops += 8.0 * std::ldexp(1.0, (int)unions[i].size());
        have[n] = 1;
        val[a] = Tensor();
        val[b] = Tensor();
    }
    // Circuit tensors under every node (for the folded leaves' origin).
    std::vector<std::vector<int>> under(L + M);
    for (int t = 0; t < L; ++t) under[t] = plan->net.origin[t];
    for (int i = 0; i < M; ++i) {
        under[L + i] = under[plan->tree[i].a];
        under[L + i].insert(under[L + i].end(), under[plan->tree[i].b].begin(), under[plan->tree[i].b].end());
    }
    std::vector<Tensor> leaves;
    std::vector<std::vector<int>> leaf_idx, origin;
    std::vector<int> new_id(L + M, -1);
    for (int t = 0; t < L; ++t)
        if (!inside[t]) {
            new_id[t] = (int)leaves.size();
            leaves.push_back(plan->net.leaves[t]);
            leaf_idx.push_back(p.leaf_idx[t]);
            origin.push_back(plan->net.origin[t]);
        }
    for (int n = L; n < L + M; ++n)
        if (top[n]) {
            new_id[n] = (int)leaves.size();
            leaves.push_back(std::move(val[n]));
            leaf_idx.push_back(sets[n]);
            std::sort(under[n].begin(), under[n].end());
            origin.push_back(under[n]);
        }
    const int L2 = (int)leaves.size();
    std::vector<Merge> tree;
    for (int i = 0; i < M; ++i) {
        const int n = L + i;
        if (inside[n] || top[n]) continue;
        tree.push_back(Merge{new_id[plan->tree[i].a], new_id[plan->tree[i].b]});
        new_id[n] = L2 + (int)tree.size() - 1;
    }
    plan->info.n_folded_steps = M - (int)tree.size();
    plan->info.flops_folded = folded_flops;
    plan->net.leaves = std::move(leaves);
    plan->net.origin = std::move(origin);
    p.leaf_idx = std::move(leaf_idx);
    plan->tree = std::move(tree);
}

// Runs f(0..n-1) on up to 16 host threads.  Each trial writes only its own
// result slot and the caller scans the slots in index order, so the plan does
// not depend on the thread count or scheduling.
template <class F>
static void parallel_trials(int n, F f) {
    const int hw = (int)std::thread::hardware_concurrency();
    const int nt = std::max(1, std::min({n, hw > 0 ? hw : 1, 16}));
    if (nt == 1) {
        for (int t = 0; t < n; ++t) f(t);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> pool;
    for (int w = 0; w < nt; ++w)
        pool.emplace_back([&]() {
            for (int t = next++; t < n; t = next++) f(t);
        });
    for (auto &th : pool) th.join();
}

// The search's result before folding: tree, slice set, dynamic leaves and
// its per-pair cost under the problem's weight.
struct SearchResult {
    std::vector<Merge> tree;
    std::vector<int> sliced;
    std::vector<char> dyn;
    double score = 0;
};

static bool search_once(qc_plan *plan, const OrderProblem &p, const qc_slice_spec *spec, std::string &err,
                        SearchResult &out) {
    const int k_target = spec ? spec->log2_slices : 0;
    const double cap = spec ? spec->log2_max_entries : 0;
    const int trials = spec ? std::max(1, spec->greedy_trials) : 1;
    const uint64_t seed = spec ? spec->seed : 0;
    const bool quick = spec && spec->quick;   // no subtree reconfiguration
    std::vector<char> sliceable(p.n_index, 0);
    for (const auto &li : p.leaf_idx)
        for (int e : li) sliceable[e] = !p.kept(e);   // summed indices only (fixed outputs are not in leaf_idx)
    std::vector<int> explicit_s;
    if (spec && spec->n_explicit > 0) {
        for (int i = 0; i < spec->n_explicit; ++i) {
            const int q = spec->explicit_segments[2 * i], o = spec->explicit_segments[2 * i + 1];
            const int e = plan->net.find_segment(q, o);
            if (e < 0 || !sliceable[e] || plan->net.out_qubit[e] >= 0 || o == 0) {
                err = "explicit segment (" + std::to_string(q) + "," + std::to_string(o) + ") cannot be sliced";
                return false;
            }
            if (std::count(explicit_s.begin(), explicit_s.end(), e)) { err = "repeated explicit segment"; return false; }
            explicit_s.push_back(e);
        }
        if (k_target >= 0 && k_target < spec->n_explicit) { err = "log2_slices below the number of explicit segments"; return false; }
    }
    const int kt = k_target < 0 ? 0 : k_target;
    bool have = false;
    double best_total = 0, best_ach = 1e9;
    std::vector<Merge> best_tree;
    std::vector<int> best_sliced;
    double last_ach = 0;
    std::vector<char> none(p.n_index, 0);
    for (int e : explicit_s) none[e] = 1;
    struct Trial {
        std::vector<Merge> tree;
        std::vector<int> sl;
        double ach = 0, total = 0;
        bool ok = false;
    };
    std::vector<Trial> tr(trials);
    // Leaves holding an output segment (or a caller-chosen slice) differ per
    // (slice, bitstring); the rest can be folded.
    std::vector<char> dyn0(p.leaf_idx.size(), 0);
    for (size_t t = 0; t < p.leaf_idx.size(); ++t)
        for (int e : plan->net.leaves[t].idx)
            if (plan->net.out_qubit[e] >= 0 || none[e]) dyn0[t] = 1;
    parallel_trials(trials, [&](int t) {
        Trial &r = tr[t];
        r.tree = greedy_order(p, none, seed + 0x1000 * t, t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8));
        if (!quick) reconfigure(p, r.tree, none, dyn0, 0, seed + 0x3000 + t, 2);
        r.sl = explicit_s;
        r.ok = choose_slices(p, r.tree, kt, cap, r.sl, sliceable, r.ach);
        if (r.ok) {
            std::vector<char> rm(p.n_index, 0);
            for (int e : r.sl) rm[e] = 1;
            r.total = tree_cost(p, r.tree, rm).flops * std::ldexp(1.0, (int)r.sl.size());
        }
    });
    std::vector<int> ok_trials;
    for (int t = 0; t < trials; ++t) {
        Trial &r = tr[t];
        last_ach = std::min(last_ach == 0 ? r.ach : last_ach, r.ach);
        if (!r.ok) { best_ach = std::min(best_ach, r.ach); continue; }
        ok_trials.push_back(t);
        if (!have || r.sl.size() < best_sliced.size() || (r.sl.size() == best_sliced.size() && r.total < best_total)) {
            have = true; best_total = r.total; best_tree = r.tree; best_sliced = r.sl;
        }
    }
    if (!have) {
        int n_sliceable = 0;
        for (char c : sliceable) n_sliceable += c;
        if (kt > n_sliceable)
            err = "asked for " + std::to_string(kt) + " slice bits but the simplified network has only " +
                  std::to_string(n_sliceable) + " sliceable indices";
        else
            err = "cannot meet a cap of 2^" + std::to_string(cap) + " entries; smallest largest-intermediate found 2^" +
                  std::to_string(best_ach);
        return false;
    }
    // The first-stage cost (unfolded flops of the first order) ranks
    // candidates only roughly: the best few slice sets with the fewest slices
    // each go through the re-search of the order on the sliced network and
    // the constant-first orders, and the one with the least per-slice device
    // work wins (ties: first in trial order).
    std::stable_sort(ok_trials.begin(), ok_trials.end(), [&](int x, int y) {
        if (tr[x].sl.size() != tr[y].sl.size()) return tr[x].sl.size() < tr[y].sl.size();
        return tr[x].total < tr[y].total;
    });
    const size_t n_cand = std::min<size_t>(ok_trials.size(), 8);
    std::vector<std::vector<int>> slices_of_cand(n_cand);
    for (size_t ci = 0; ci < n_cand; ++ci) slices_of_cand[ci] = tr[ok_trials[ci]].sl;
    // The candidates are refined in parallel, each into its own slot, and
    // compared in candidate order afterwards (so the plan does not depend on
    // the thread count).
    struct Refined {
        bool ok = false;
        double dev = 0;
        std::vector<Merge> tree;
        std::vector<char> dyn;
    };
    std::vector<Refined> refined(n_cand);
    parallel_trials((int)n_cand, [&](int cii) {
        const size_t ci = (size_t)cii;
        const Trial &cand = tr[ok_trials[ci]];
        if (cand.sl.size() != tr[ok_trials[0]].sl.size()) return;
        std::vector<Merge> tree = cand.tree;
        std::vector<char> rm(p.n_index, 0);
        for (int e : cand.sl) rm[e] = 1;
        // A second slice set for this tree: one index at a time, the tree
        // reconfigured for the sliced network after each, so that it can
        // gather its expensive merges on the sliced indices.  Kept if its
        // per-slice work beats the first set's once both are reconfigured.
        if (!quick) {
            std::vector<Merge> t2 = cand.tree;
            std::vector<int> sl2 = explicit_s;
            std::vector<char> rm2(p.n_index, 0);
            for (int e : sl2) rm2[e] = 1;
            double ach = 0;
            bool done = false;
            for (int step = 0; step < 64 && !done; ++step) {
                done = choose_slices(p, t2, kt, cap, sl2, sliceable, ach, 1);
                std::fill(rm2.begin(), rm2.end(), 0);
                for (int e : sl2) rm2[e] = 1;
                std::vector<char> dyn2(p.leaf_idx.size(), 0);
                for (size_t t = 0; t < p.leaf_idx.size(); ++t)
                    for (int e : plan->net.leaves[t].idx)
                        if (plan->net.out_qubit[e] >= 0 || rm2[e]) dyn2[t] = 1;
                reconfigure(p, t2, rm2, dyn2, 0, seed + 0xB000 + 0x100 * ci + step, 2);
            }
            if (done && (int)sl2.size() == (int)cand.sl.size()) {
                std::vector<char> dyn2(p.leaf_idx.size(), 0), dyn1(p.leaf_idx.size(), 0);
                for (size_t t = 0; t < p.leaf_idx.size(); ++t)
                    for (int e : plan->net.leaves[t].idx) {
                        if (plan->net.out_qubit[e] >= 0 || rm2[e]) dyn2[t] = 1;
                        if (plan->net.out_qubit[e] >= 0 || rm[e]) dyn1[t] = 1;
                    }
                std::vector<Merge> t1 = tree;
                const double f2 = reconfigure(p, t2, rm2, dyn2, cap, seed + 0xC000 + ci, 2);
                const double f1 = reconfigure(p, t1, rm, dyn1, cap, seed + 0xD000 + ci, 2);
                const TreeCost c2 = tree_cost(p, t2, rm2);
                if (f2 < f1 && (cap <= 0 || c2.max_log2 <= cap)) {
                    tree = t2;
                    rm = rm2;
                    slices_of_cand[ci] = sl2;
                } else {
                    tree = t1;
                }
            }
        }
        // Re-search the order on the sliced network; keep it if cheaper and
        // still within the cap.
        TreeCost bc = tree_cost(p, tree, rm);
        std::vector<std::pair<std::vector<Merge>, TreeCost>> re(trials);
        parallel_trials(trials, [&](int t) {
            re[t].first = greedy_order(p, rm, seed + 0x9000 + 0x1000 * t + 0x100000 * ci,
                                       t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8));
            re[t].second = tree_cost(p, re[t].first, rm);
        });
        for (auto &r : re)
            if ((cap <= 0 || r.second.max_log2 <= cap) && r.second.flops < bc.flops) { bc = r.second; tree = r.first; }
        // Pair-invariant work: a leaf is dynamic if it holds a sliced or an
        // output segment; every other subtree has the same value for all
        // (slice, bitstring) pairs.  Constant-first orders, keeping the one
        // with the least per-pair work.
        std::vector<char> dyn_leaf(p.leaf_idx.size(), 0);
        for (size_t t = 0; t < p.leaf_idx.size(); ++t)
            for (int e : plan->net.leaves[t].idx)
                if (plan->net.out_qubit[e] >= 0 || rm[e]) dyn_leaf[t] = 1;
        double dev = per_pair_cost(p, tree, rm, dyn_leaf);
        const int const_cap = std::max(4, (int)bc.max_log2);
        std::vector<std::pair<std::vector<Merge>, double>> ph(trials);
        parallel_trials(trials, [&](int t) {
            ph[t].first = greedy_order_phased(p, rm, seed + 0x5000 + 0x1000 * t + 0x100000 * ci,
                                              t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8), &dyn_leaf, const_cap);
            const TreeCost c = tree_cost(p, ph[t].first, rm);
            ph[t].second = (cap > 0 && c.max_log2 > cap) ? -1.0 : per_pair_cost(p, ph[t].first, rm, dyn_leaf);
        });
        for (auto &r : ph)
            if (r.second >= 0 && r.second < dev) { dev = r.second; tree = r.first; }
        // Local optimisation of the chosen tree for this slice set.
        if (!quick) dev = reconfigure(p, tree, rm, dyn_leaf, cap, seed + 0x7000 + ci, kReconfSweeps);
        refined[ci].ok = true;
        refined[ci].dev = dev;
        refined[ci].tree = std::move(tree);
        refined[ci].dyn = std::move(dyn_leaf);
    });
    double best_score = -1;
    std::vector<char> best_dyn;
    for (size_t ci = 0; ci < n_cand; ++ci) {
        if (!refined[ci].ok) continue;
        if (best_score < 0 || refined[ci].dev < best_score) {
            best_score = refined[ci].dev;
            best_tree = refined[ci].tree;
            best_sliced = slices_of_cand[ci];
            best_dyn = refined[ci].dyn;
        }
    }
    (void)last_ach;
    out.tree = std::move(best_tree);
    out.sliced = std::move(best_sliced);
    out.dyn = std::move(best_dyn);
    out.score = best_score;
    return true;
}

bool search_plan(qc_plan *plan, const qc_slice_spec *spec, std::string &err) {
    const OrderProblem &p = plan->prob;
    SearchResult best;
    if (!search_once(plan, p, spec, err, best)) return false;
    if (!(spec && spec->quick)) {
        // The same search under the second weight, kept if its tree costs
        // less per pair under the first weight's step cost.
        OrderProblem alt = p;
        alt.move_per_mac = kMovePerMacAlt;
        SearchResult r;
        std::string err2;
        if (search_once(plan, alt, spec, err2, r)) {
            std::vector<char> rm(p.n_index, 0);
            for (int e : r.sliced) rm[e] = 1;
            if (r.sliced.size() == best.sliced.size() && per_pair_cost(p, r.tree, rm, r.dyn) < best.score)
                best = std::move(r);
        }
    }
    std::vector<Merge> best_tree = std::move(best.tree);
    std::vector<int> best_sliced = std::move(best.sliced);
    std::vector<char> dyn_leaf = std::move(best.dyn);
    {
        const TreeCost c0 = tree_cost(p, best_tree, std::vector<char>(p.n_index, 0));
        plan->info.flops_unsliced = c0.flops;
    }
    plan->tree = best_tree;
    plan->sliced = best_sliced;
    plan->tree_full = best_tree;
    plan->origin_full = plan->net.origin;
    fold_invariant_subtrees(plan, dyn_leaf);
    std::vector<char> rm2(plan->prob.n_index, 0);
    for (int e : plan->sliced) rm2[e] = 1;
    const TreeCost cf = tree_cost(plan->prob, plan->tree, rm2);
    plan->info.log2_slices = (int)best_sliced.size();
    plan->info.log2_max_entries = cf.max_log2;
    plan->info.flops_per_slice = cf.flops;
    plan->info.bytes_per_slice = cf.bytes;
    plan->info.peak_live_bytes = cf.peak_live;
    return true;
}

}  // namespace qc
