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
            else {  // shared: stays if another live tensor holds it
                if (holders[A[i]].size() > 2) ++r;
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
            if (!(both && holders[e].size() == 2)) c.push_back(e);
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
                          double &achieved_log2) {
    std::vector<char> removed(p.n_index, 0);
    for (int e : sliced) removed[e] = 1;
    for (;;) {
        std::vector<std::vector<int>> sets, unions;
        node_sets(p, tree, removed, sets, unions);
        int maxr = 0;
        for (auto &s : sets) maxr = std::max(maxr, (int)s.size());
        achieved_log2 = maxr;
        const bool cap_ok = cap_log2 <= 0 || maxr <= cap_log2;
        if (cap_ok && (int)sliced.size() >= k_target) return true;
        // Candidates: indices of the largest nodes.
        std::vector<char> cand(p.n_index, 0);
        for (auto &s : sets)
            if ((int)s.size() == maxr)
                for (int e : s) cand[e] = sliceable[e] && !removed[e];
        int best = -1;
        int best_max = 1 << 30;
        double best_flops = 0;
        for (int e = 0; e < p.n_index; ++e) {
            if (!cand[e]) continue;
            int m = 0;
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
static double per_pair_flops(const OrderProblem &p, const std::vector<Merge> &tree,
                             const std::vector<char> &removed, const std::vector<char> &dyn_leaf) {
    std::vector<std::vector<int>> sets, unions;
    node_sets(p, tree, removed, sets, unions);
    const int L = (int)p.leaf_idx.size();
    std::vector<char> dyn(dyn_leaf.begin(), dyn_leaf.end());
    double f = 0;
    for (size_t i = 0; i < tree.size(); ++i) {
        const bool d = dyn[tree[i].a] || dyn[tree[i].b];
        dyn.push_back(d);
        if (d || (int)sets[L + i].size() > kFoldMaxLog2) f += 8.0 * std::ldexp(1.0, (int)unions[i].size());
    }
    return f;
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

bool search_plan(qc_plan *plan, const qc_slice_spec *spec, std::string &err) {
    const OrderProblem &p = plan->prob;
    const int k_target = spec ? spec->log2_slices : 0;
    const double cap = spec ? spec->log2_max_entries : 0;
    const int trials = spec ? std::max(1, spec->greedy_trials) : 1;
    const uint64_t seed = spec ? spec->seed : 0;
    std::vector<char> sliceable(p.n_index, 0);
    for (const auto &li : p.leaf_idx)
        for (int e : li) sliceable[e] = 1;   // summed indices only (outputs are not in leaf_idx)
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
    parallel_trials(trials, [&](int t) {
        Trial &r = tr[t];
        r.tree = greedy_order(p, none, seed + 0x1000 * t, t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8));
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
    double best_score = -1;
    std::vector<char> best_dyn;
    for (size_t ci = 0; ci < n_cand; ++ci) {
        const Trial &cand = tr[ok_trials[ci]];
        if (cand.sl.size() != tr[ok_trials[0]].sl.size()) break;
        std::vector<Merge> tree = cand.tree;
        std::vector<char> rm(p.n_index, 0);
        for (int e : cand.sl) rm[e] = 1;
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
        double dev = per_pair_flops(p, tree, rm, dyn_leaf);
        const int const_cap = std::max(4, (int)bc.max_log2);
        std::vector<std::pair<std::vector<Merge>, double>> ph(trials);
        parallel_trials(trials, [&](int t) {
            ph[t].first = greedy_order_phased(p, rm, seed + 0x5000 + 0x1000 * t + 0x100000 * ci,
                                              t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8), &dyn_leaf, const_cap);
            const TreeCost c = tree_cost(p, ph[t].first, rm);
            ph[t].second = (cap > 0 && c.max_log2 > cap) ? -1.0 : per_pair_flops(p, ph[t].first, rm, dyn_leaf);
        });
        for (auto &r : ph)
            if (r.second >= 0 && r.second < dev) { dev = r.second; tree = r.first; }
        if (best_score < 0 || dev < best_score) {
            best_score = dev;
            best_tree = tree;
            best_sliced = cand.sl;
            best_dyn = dyn_leaf;
        }
    }
    std::vector<char> dyn_leaf = best_dyn;
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
    (void)last_ach;
    return true;
}

}  // namespace qc
