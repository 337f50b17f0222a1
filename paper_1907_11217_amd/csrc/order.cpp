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
#include <cmath>
#include <queue>

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
    auto push = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        const double sa = std::ldexp(1.0, (int)sets[a].size()), sb = std::ldexp(1.0, (int)sets[b].size());
        double key = std::ldexp(1.0, result_rank(a, b)) - sa - sb;
        if (temperature > 0) key -= temperature * (sa + sb) * rng.gumbel();
        heap.push(Cand{key, a, b});
    };
    for (int e = 0; e < p.n_index; ++e)
        for (size_t i = 0; i < holders[e].size(); ++i)
            for (size_t j = i + 1; j < holders[e].size(); ++j) push(holders[e][i], holders[e][j]);

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
        tree.push_back(Merge{a, b});
        --n_alive;
        return id;
    };
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
    for (int t = 0; t < trials; ++t) {
        std::vector<Merge> tree = greedy_order(p, none, seed + 0x1000 * t, t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8));
        std::vector<int> sl = explicit_s;
        double ach = 0;
        const bool ok = choose_slices(p, tree, kt, cap, sl, sliceable, ach);
        last_ach = std::min(last_ach == 0 ? ach : last_ach, ach);
        if (!ok) { best_ach = std::min(best_ach, ach); continue; }
        std::vector<char> rm(p.n_index, 0);
        for (int e : sl) rm[e] = 1;
        const TreeCost c = tree_cost(p, tree, rm);
        const double total = c.flops * std::ldexp(1.0, (int)sl.size());
        if (!have || sl.size() < best_sliced.size() || (sl.size() == best_sliced.size() && total < best_total)) {
            have = true; best_total = total; best_tree = tree; best_sliced = sl;
        }
    }
    if (!have) {
        err = "cannot meet a cap of 2^" + std::to_string(cap) + " entries; smallest largest-intermediate found 2^" +
              std::to_string(best_ach);
        return false;
    }
    // Re-search the order on the sliced network; keep it if it is cheaper
    // and still within the cap.
    std::vector<char> rm(p.n_index, 0);
    for (int e : best_sliced) rm[e] = 1;
    TreeCost bc = tree_cost(p, best_tree, rm);
    for (int t = 0; t < trials; ++t) {
        std::vector<Merge> tree = greedy_order(p, rm, seed + 0x9000 + 0x1000 * t, t == 0 ? 0.0 : 0.1 + 0.05 * (t % 8));
        const TreeCost c = tree_cost(p, tree, rm);
        if ((cap <= 0 || c.max_log2 <= cap) && c.flops < bc.flops) { bc = c; best_tree = tree; }
    }
    plan->tree = best_tree;
    plan->sliced = best_sliced;
    const TreeCost c0 = tree_cost(p, best_tree, std::vector<char>(p.n_index, 0));
    plan->info.log2_slices = (int)best_sliced.size();
    plan->info.log2_max_entries = bc.max_log2;
    plan->info.flops_per_slice = bc.flops;
    plan->info.bytes_per_slice = bc.bytes;
    plan->info.flops_unsliced = c0.flops;
    plan->info.peak_live_bytes = bc.peak_live;
    (void)last_ach;
    return true;
}

}  // namespace qc
