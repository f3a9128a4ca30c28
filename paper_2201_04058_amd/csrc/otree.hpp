// Overlap Tree (Sec. 3.3) and the cache replacement policies of Sec. 3.4
// (Algorithm 1 and its baselines).  Host only.
#pragma once

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace atp {

// A generalised suffix tree of metapath strings (Sec. 3.3, "The structure"):
// every inserted metapath gets a terminator symbol of its own, so each of its
// suffixes ends in a leaf; an internal node is an overlap of at least two
// suffixes.  Node frequency f counts the inserted suffixes that pass through
// the node, i.e. the occurrences of its string in the workload (f = 1 at
// leaves).  Each node carries a constraints index (Sec. 3.3, "Handling
// constrained queries"): constraint key -> per-key frequency and cache slot.
class OverlapTree {
public:
    struct KeyEntry {
        int64_t f = 0;        // occurrences of (string, constraints)
        int64_t item = -1;    // cache item id, -1 if not cached
        double cost = 0;      // time to compute (last measured), seconds
        double nnz = 0;       // nonzeros of the result (last seen)
    };
    struct Node {
        std::vector<int32_t> label;  // symbols on the edge from the parent
        int parent = -1;
        std::map<int32_t, int> children;  // first symbol -> child
        int64_t f = 0;
        int depth = 0;                    // length of the node's string (terminators included)
        std::map<std::string, KeyEntry> keys;
        bool leaf() const { return children.empty(); }
    };

    OverlapTree();
    // Insert symbols (non-negative) and all their suffixes; a fresh terminator
    // is appended.  Returns the terminator used.
    int32_t insert(const std::vector<int32_t> &symbols);
    // Node whose string equals `s` (a string ending inside an edge has no
    // node: returns -1), and the node reached, even mid-edge (the deeper node).
    int find(const std::vector<int32_t> &s) const;
    // occurrences of s as a substring of inserted strings (0 if absent)
    int64_t frequency(const std::vector<int32_t> &s) const;
    const Node &node(int i) const { return nodes_[i]; }
    Node &node(int i) { return nodes_[i]; }
    int size() const { return (int)nodes_.size(); }
    int64_t leaves() const;
    int64_t lambda() const { return lambda_; }
    // every node strictly below `v`
    void for_subtree(int v, const std::function<void(int)> &fn) const;

private:
    std::vector<Node> nodes_;
    int32_t next_term_ = -1;
    int64_t lambda_ = 0;  // total symbols inserted (without terminators)
    void insert_suffix(const std::vector<int32_t> &s, size_t from);
};

// Replacement policies over cache items with size s, cost c and frequency f.
enum class Policy { Otree = 1, Pgds = 2, Lru = 3 };

// Cache bookkeeping (no payload): Algorithm 1 ("Atrapos-OTree": PGDS utility
// h = f*c/s + L with inflation L, and on insertion / eviction of an item the
// cost of the cached items in its Overlap-Tree subtree is decreased /
// reinstated), plain PGDS, and LRU.  Items larger than 80% of the budget are
// never admitted (Sec. 4.1, "Evaluation Setting").
class CachePolicy {
public:
    struct Item {
        double size = 0, cost = 0;
        int64_t f = 0;
        double l = 0;   // inflation value when last inserted / hit
        double h = 0;   // utility
        int64_t tick = 0;
        bool cached = false;
    };
    CachePolicy(Policy p, double budget) : policy_(p), budget_(budget) {}
    // descendants(item) lists the items in the item's Overlap-Tree subtree
    void set_subtree_fn(std::function<std::vector<int64_t>(int64_t)> fn) { subtree_ = std::move(fn); }
    // New item id (not cached yet).
    int64_t add_item(double size, double cost);
    // A request of an item (Algorithm 1's loop body): a hit refreshes it; a
    // miss tries to insert it, evicting by the policy.  Returns whether it is
    // cached afterwards; evicted items are appended to `evicted`.
    bool request(int64_t id, std::vector<int64_t> &evicted);
    // bookkeeping of a hit without insertion attempt (DP reuse)
    void touch(int64_t id);
    void drop(int64_t id);  // forget a cached item (payload freed outside)
    const Item &item(int64_t id) const { return items_.at(id); }
    double used() const { return used_; }
    double budget() const { return budget_; }
    double inflation() const { return L_; }
    int64_t cached_count() const;

private:
    Policy policy_;
    double budget_, used_ = 0, L_ = 0;
    int64_t tick_ = 0;
    std::map<int64_t, Item> items_;
    std::function<std::vector<int64_t>(int64_t)> subtree_;
    void utility(Item &it) const;
    int64_t victim() const;
};

}  // namespace atp
