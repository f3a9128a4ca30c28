// Overlap Tree (Sec. 3.3) and cache replacement policies (Sec. 3.4).
#include "otree.hpp"

#include <algorithm>
#include <limits>

namespace atp {

OverlapTree::OverlapTree() { nodes_.emplace_back(); }

int32_t OverlapTree::insert(const std::vector<int32_t> &symbols) {
    std::vector<int32_t> s(symbols);
    const int32_t term = next_term_--;
    s.push_back(term);
    for (size_t k = 0; k + 1 < s.size(); ++k) insert_suffix(s, k);
    lambda_ += (int64_t)symbols.size();
    return term;
}

// Walk from the root along s[from..]; count the suffix in every node it
// passes; where the walk leaves the tree create a leaf, splitting an edge if
// the mismatch falls inside it.  The terminator is unique, so every suffix
// ends in a new leaf.
void OverlapTree::insert_suffix(const std::vector<int32_t> &s, size_t from) {
    int v = 0;
    size_t pos = from;
    while (true) {
        auto it = nodes_[v].children.find(s[pos]);
        if (it == nodes_[v].children.end()) {
            Node leaf;
            leaf.label.assign(s.begin() + pos, s.end());
            leaf.parent = v;
            leaf.f = 1;
            leaf.depth = nodes_[v].depth + (int)leaf.label.size();
            nodes_.push_back(std::move(leaf));
            nodes_[v].children[s[pos]] = (int)nodes_.size() - 1;
            return;
        }
        const int ch = it->second;
        size_t m = 0;
        {
            const std::vector<int32_t> &lab = nodes_[ch].label;
            while (m < lab.size() && pos + m < s.size() && lab[m] == s[pos + m]) ++m;
            if (m == lab.size()) {
                nodes_[ch].f += 1;
                v = ch;
                pos += m;
                continue;
            }
        }
        // split the edge to ch after m symbols
        Node mid;
        mid.label.assign(nodes_[ch].label.begin(), nodes_[ch].label.begin() + m);
        mid.parent = v;
        mid.depth = nodes_[v].depth + (int)m;
        mid.f = nodes_[ch].f + 1;
        const int mid_id = (int)nodes_.size();
        nodes_.push_back(std::move(mid));
        Node &chn = nodes_[ch];
        const int32_t first_rest = chn.label[m];
        // a leaf whose remaining label is only its terminator stood for a whole
        // metapath; that string is now the internal node's, so its keys move
        if (chn.label.size() == m + 1 && chn.label[m] < 0 && chn.leaf()) {
            nodes_[mid_id].keys = std::move(chn.keys);
            chn.keys.clear();
        }
        chn.label.erase(chn.label.begin(), chn.label.begin() + m);
        chn.parent = mid_id;
        nodes_[mid_id].children[first_rest] = ch;
        nodes_[v].children[s[pos]] = mid_id;
        Node leaf;
        leaf.label.assign(s.begin() + pos + m, s.end());
        leaf.parent = mid_id;
        leaf.f = 1;
        leaf.depth = nodes_[mid_id].depth + (int)leaf.label.size();
        nodes_.push_back(std::move(leaf));
        nodes_[mid_id].children[s[pos + m]] = (int)nodes_.size() - 1;
        return;
    }
}

// The node standing for string s: an explicit node whose string is s, or a
// leaf whose string is s followed by its terminator (a whole metapath).
int OverlapTree::find(const std::vector<int32_t> &s) const {
    int v = 0;
    size_t pos = 0;
    while (pos < s.size()) {
        auto it = nodes_[v].children.find(s[pos]);
        if (it == nodes_[v].children.end()) return -1;
        const int ch = it->second;
        const std::vector<int32_t> &lab = nodes_[ch].label;
        size_t m = 0;
        while (m < lab.size() && pos + m < s.size() && lab[m] == s[pos + m]) ++m;
        if (m == lab.size()) {
            v = ch;
            pos += m;
            continue;
        }
        if (pos + m < s.size()) return -1;
        // s ends inside this edge
        return (lab.size() == m + 1 && lab[m] < 0) ? ch : -1;
    }
    return v == 0 ? -1 : v;
}

int64_t OverlapTree::frequency(const std::vector<int32_t> &s) const {
    int v = 0;
    size_t pos = 0;
    while (pos < s.size()) {
        auto it = nodes_[v].children.find(s[pos]);
        if (it == nodes_[v].children.end()) return 0;
        const int ch = it->second;
        const std::vector<int32_t> &lab = nodes_[ch].label;
        size_t m = 0;
        while (m < lab.size() && pos + m < s.size() && lab[m] == s[pos + m]) ++m;
        if (pos + m == s.size()) return nodes_[ch].f;
        if (m < lab.size()) return 0;
        v = ch;
        pos += m;
    }
    return v == 0 ? 0 : nodes_[v].f;
}

int64_t OverlapTree::leaves() const {
    int64_t n = 0;
    for (size_t i = 1; i < nodes_.size(); ++i) n += nodes_[i].leaf();
    return n;
}

void OverlapTree::for_subtree(int v, const std::function<void(int)> &fn) const {
    std::vector<int> stack;
    for (auto &kv : nodes_[v].children) stack.push_back(kv.second);
    while (!stack.empty()) {
        int u = stack.back();
        stack.pop_back();
        fn(u);
        for (auto &kv : nodes_[u].children) stack.push_back(kv.second);
    }
}

// ---------------------------------------------------------------------------

int64_t CachePolicy::add_item(double size, double cost) {
    const int64_t id = items_.empty() ? 0 : items_.rbegin()->first + 1;
    Item it;
    it.size = size;
    it.cost = cost;
    items_[id] = it;
    return id;
}

void CachePolicy::utility(Item &it) const {
    it.h = (it.size > 0 ? (double)it.f * it.cost / it.size : 0.0) + it.l;
}

int64_t CachePolicy::victim() const {
    int64_t best = -1;
    double bh = std::numeric_limits<double>::infinity();
    int64_t bt = std::numeric_limits<int64_t>::max();
    for (const auto &kv : items_) {
        const Item &it = kv.second;
        if (!it.cached) continue;
        if (policy_ == Policy::Lru) {
            if (it.tick < bt) {
                bt = it.tick;
                best = kv.first;
            }
        } else if (it.h < bh) {  // ties: the smallest id
            bh = it.h;
            best = kv.first;
        }
    }
    return best;
}

int64_t CachePolicy::cached_count() const {
    int64_t n = 0;
    for (const auto &kv : items_) n += kv.second.cached;
    return n;
}

void CachePolicy::touch(int64_t id) {
    std::vector<int64_t> ev;
    request(id, ev);
}

void CachePolicy::drop(int64_t id) {
    auto it = items_.find(id);
    if (it == items_.end() || !it->second.cached) return;
    it->second.cached = false;
    used_ -= it->second.size;
}

bool CachePolicy::request(int64_t id, std::vector<int64_t> &evicted) {
    Item &p = items_.at(id);
    p.f += 1;
    p.tick = ++tick_;
    if (p.cached) {  // hit: refresh the utility with the current inflation
        p.l = L_;
        utility(p);
        return true;
    }
    if (p.size > 0.8 * budget_) return false;
    while (used_ + p.size > budget_) {
        const int64_t v = victim();
        if (v < 0) return false;
        Item &q = items_.at(v);
        if (policy_ != Policy::Lru) L_ = q.h;
        q.cached = false;
        used_ -= q.size;
        evicted.push_back(v);
        if (policy_ == Policy::Otree && subtree_) {
            for (int64_t e : subtree_(v)) {  // reinstate q's cost in its subtree
                auto ie = items_.find(e);
                if (ie == items_.end() || !ie->second.cached) continue;
                ie->second.cost += q.cost;
                utility(ie->second);
            }
        }
    }
    p.cached = true;
    used_ += p.size;
    p.l = L_;
    utility(p);
    if (policy_ == Policy::Otree && subtree_) {
        for (int64_t e : subtree_(id)) {  // the subtree is cheaper to recompute given p
            auto ie = items_.find(e);
            if (ie == items_.end() || !ie->second.cached) continue;
            ie->second.cost -= p.cost;
            utility(ie->second);
        }
    }
    return true;
}

}  // namespace atp

// ---------------------------------------------------------------------------
// C-ABI of the standalone objects

#include "../../include/atrapos.h"

struct atp_otree {
    atp::OverlapTree tree;
};

extern "C" {

atp_status atp_otree_create(atp_otree **out) {
    if (!out) return ATP_EINVAL;
    *out = new atp_otree();
    return ATP_OK;
}

atp_status atp_otree_destroy(atp_otree *t) {
    if (!t) return ATP_EINVAL;
    delete t;
    return ATP_OK;
}

atp_status atp_otree_insert(atp_otree *t, const int32_t *symbols, int32_t n) {
    if (!t || !symbols || n < 1) return ATP_EINVAL;
    for (int32_t i = 0; i < n; ++i)
        if (symbols[i] < 0) return ATP_EINVAL;
    t->tree.insert(std::vector<int32_t>(symbols, symbols + n));
    return ATP_OK;
}

atp_status atp_otree_frequency(const atp_otree *t, const int32_t *symbols, int32_t n, int64_t *f) {
    if (!t || !f || n < 0 || (n > 0 && !symbols)) return ATP_EINVAL;
    *f = n == 0 ? 0 : t->tree.frequency(std::vector<int32_t>(symbols, symbols + n));
    return ATP_OK;
}

atp_status atp_otree_shape(const atp_otree *t, int64_t *nodes, int64_t *leaves, int64_t *lambda,
                           int64_t *thin_internal, int64_t *leaves_f_not_1) {
    if (!t) return ATP_EINVAL;
    const atp::OverlapTree &tr = t->tree;
    int64_t thin = 0, bad = 0;
    for (int i = 1; i < tr.size(); ++i) {
        const auto &nd = tr.node(i);
        if (nd.leaf())
            bad += nd.f != 1;
        else
            thin += nd.children.size() < 2;
    }
    if (nodes) *nodes = tr.size();
    if (leaves) *leaves = tr.leaves();
    if (lambda) *lambda = tr.lambda();
    if (thin_internal) *thin_internal = thin;
    if (leaves_f_not_1) *leaves_f_not_1 = bad;
    return ATP_OK;
}

atp_status atp_cache_simulate(int32_t policy, double budget, int32_t n_items, const double *size, const double *cost,
                              const int32_t *parent, int32_t n_req, const int32_t *req, int32_t *hit,
                              int32_t *cached_after, int32_t *final_cached) {
    if (n_items < 0 || n_req < 0 || (n_items > 0 && (!size || !cost)) || (n_req > 0 && !req)) return ATP_EINVAL;
    if (policy != ATP_CACHE_OTREE && policy != ATP_CACHE_PGDS && policy != ATP_CACHE_LRU) return ATP_EINVAL;
    const atp::Policy pol = policy == ATP_CACHE_OTREE ? atp::Policy::Otree
                            : policy == ATP_CACHE_PGDS ? atp::Policy::Pgds
                                                       : atp::Policy::Lru;
    atp::CachePolicy cp(pol, budget);
    for (int32_t i = 0; i < n_items; ++i) cp.add_item(size[i], cost[i]);
    // descendants through the parent links
    std::vector<std::vector<int64_t>> desc(n_items);
    for (int32_t i = 0; i < n_items; ++i) {
        int32_t p = parent ? parent[i] : -1;
        int guard = 0;
        while (p >= 0 && p < n_items && guard++ <= n_items) {
            desc[p].push_back(i);
            p = parent[p];
        }
    }
    cp.set_subtree_fn([&](int64_t id) { return desc[id]; });
    for (int32_t r = 0; r < n_req; ++r) {
        const int32_t id = req[r];
        if (id < 0 || id >= n_items) return ATP_EINVAL;
        const bool before = cp.item(id).cached;
        std::vector<int64_t> ev;
        const bool after = cp.request(id, ev);
        if (hit) hit[r] = before;
        if (cached_after) cached_after[r] = after;
    }
    if (final_cached)
        for (int32_t i = 0; i < n_items; ++i) final_cached[i] = cp.item(i).cached;
    return ATP_OK;
}

}  // extern "C"
