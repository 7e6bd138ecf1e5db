// Guide tree of a family from its pairwise distances (stage II of the
// method: weighted UPGMA on the distances of the posterior stage; Methods,
// opening paragraph) and the tree-guided distance between sequences (number
// of nodes of the smallest subtree holding both; "Selective consistency").
// Host code: O(n^2) memory and, with cached row minima, about O(n^2) time
// for the few thousand sequences of a family.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "qp.h"
#include "qp_internal.h"

namespace {

constexpr int32_t kMaxTreeSeqs = 32768;

// index of pair (i < j) in the condensed row-major order of qp_result.dist
inline int64_t pidx(int64_t i, int64_t j, int64_t n) { return i * n - i * (i + 1) / 2 + (j - i - 1); }

// candidate merge: distance, then the smaller and the larger cluster id
struct Key {
    double d;
    int32_t lo, hi;
    bool operator<(const Key& o) const {
        if (d != o.d) return d < o.d;
        if (lo != o.lo) return lo < o.lo;
        return hi < o.hi;
    }
};

}  // namespace

extern "C" qp_status qp_guide_tree(const double* dist, int32_t n, int32_t* merges, double* heights) {
    if (n < 1) return qp::set_error(QP_EINVAL, "n < 1");
    if (n > kMaxTreeSeqs) return qp::set_error(QP_EINVAL, "n > 32768 sequences");
    if (n == 1) return QP_OK;
    if (!dist || !merges || !heights) return qp::set_error(QP_EINVAL, "dist, merges or heights is NULL");
    const int64_t P = (int64_t)n * (n - 1) / 2;
    for (int64_t p = 0; p < P; ++p)
        if (!std::isfinite(dist[p])) return qp::set_error(QP_EINVAL, "dist holds a value that is not finite");
    // slot s holds one active cluster; the distance of slots a < b is at
    // pidx(a, b); a merge puts the new cluster in the lower slot
    std::vector<double> d;
    std::vector<int32_t> id, best;
    std::vector<uint8_t> live;
    try {
        d.assign(dist, dist + P);
        id.resize(n);
        best.resize(n);
        live.assign(n, 1);
    } catch (const std::bad_alloc&) {
        return qp::set_error(QP_ENOMEM, "out of host memory");
    }
    auto D = [&](int32_t a, int32_t b) -> double& { return a < b ? d[pidx(a, b, n)] : d[pidx(b, a, n)]; };
    auto key = [&](int32_t a, int32_t b) {
        return Key{D(a, b), std::min(id[a], id[b]), std::max(id[a], id[b])};
    };
    // best[s]: the live partner of slot s with the smallest key
    auto scan = [&](int32_t s) {
        int32_t arg = -1;
        Key k{0.0, 0, 0};
        for (int32_t t = 0; t < n; ++t) {
            if (t == s || !live[t]) continue;
            const Key c = key(s, t);
            if (arg < 0 || c < k) {
                k = c;
                arg = t;
            }
        }
        best[s] = arg;
    };
    for (int32_t s = 0; s < n; ++s) id[s] = s;
    for (int32_t s = 0; s < n; ++s) scan(s);
    for (int32_t step = 0; step < n - 1; ++step) {
        // the globally smallest candidate is the smallest cached one
        int32_t a = -1;
        Key k{0.0, 0, 0};
        for (int32_t s = 0; s < n; ++s) {
            if (!live[s] || best[s] < 0) continue;
            const Key c = key(s, best[s]);
            if (a < 0 || c < k) {
                k = c;
                a = s;
            }
        }
        int32_t b = best[a];
        if (b < a) std::swap(a, b);
        merges[2 * step] = k.lo;
        merges[2 * step + 1] = k.hi;
        heights[step] = k.d / 2.0;
        // weighted average: both merged clusters count once, whatever their size
        for (int32_t t = 0; t < n; ++t) {
            if (!live[t] || t == a || t == b) continue;
            D(a, t) = (D(a, t) + D(b, t)) / 2.0;
        }
        live[b] = 0;
        id[a] = n + step;
        // refresh the cached minima: rows that pointed at a or b rescan, the
        // others only compare with their new distance to a
        for (int32_t t = 0; t < n; ++t) {
            if (!live[t] || t == a) continue;
            if (best[t] == a || best[t] == b)
                scan(t);
            else if (key(t, a) < key(t, best[t]))
                best[t] = a;
        }
        scan(a);
    }
    return QP_OK;
}

extern "C" qp_status qp_tree_distance(const int32_t* merges, int32_t n, int32_t* out) {
    if (n < 1) return qp::set_error(QP_EINVAL, "n < 1");
    if (n > kMaxTreeSeqs) return qp::set_error(QP_EINVAL, "n > 32768 sequences");
    if (n == 1) return QP_OK;
    if (!merges || !out) return qp::set_error(QP_EINVAL, "merges or out is NULL");
    const int64_t P = (int64_t)n * (n - 1) / 2;
    std::vector<std::vector<int32_t>> members;
    std::vector<uint8_t> used;
    try {
        members.resize(2 * (size_t)n - 1);
        used.assign(2 * (size_t)n - 1, 0);
        for (int32_t s = 0; s < n; ++s) members[s].push_back(s);
    } catch (const std::bad_alloc&) {
        return qp::set_error(QP_ENOMEM, "out of host memory");
    }
    std::fill(out, out + P, 0);
    for (int32_t step = 0; step < n - 1; ++step) {
        const int32_t a = merges[2 * step], b = merges[2 * step + 1];
        const int32_t made = n + step;
        if (a < 0 || b < 0 || a >= made || b >= made || a == b || used[a] || used[b]) {
            char msg[128];
            std::snprintf(msg, sizeof(msg), "merge %d does not join two existing, unjoined clusters", step);
            return qp::set_error(QP_EINVAL, msg);
        }
        used[a] = used[b] = 1;
        // every pair split between the two clusters meets first here
        const int32_t nodes = 2 * (int32_t)(members[a].size() + members[b].size()) - 1;
        for (int32_t x : members[a])
            for (int32_t y : members[b]) out[x < y ? pidx(x, y, n) : pidx(y, x, n)] = nodes;
        try {
            std::vector<int32_t>& m = members[made];
            m.reserve(members[a].size() + members[b].size());
            m.insert(m.end(), members[a].begin(), members[a].end());
            m.insert(m.end(), members[b].begin(), members[b].end());
        } catch (const std::bad_alloc&) {
            return qp::set_error(QP_ENOMEM, "out of host memory");
        }
        std::vector<int32_t>().swap(members[a]);
        std::vector<int32_t>().swap(members[b]);
    }
    return QP_OK;
}
