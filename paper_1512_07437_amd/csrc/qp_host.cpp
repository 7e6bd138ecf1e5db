// Host memory of results.  A result and all of its arrays live in one host
// block.  Blocks of a useful size are pinned (page-locked), so the device
// writes the arrays by DMA with no bounce copy and no page faults on first
// touch, and they are recycled: a freed result's block goes to an idle pool
// and the next result of a similar size takes it instead of pinning fresh
// memory.  Small results, and results that would take the pinned total over
// its cap, use ordinary heap memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "qp.h"
#include "qp_internal.h"

namespace {

constexpr size_t kAlign = 256;                   // each array starts on this boundary
constexpr size_t kGrain = (size_t)2 << 20;       // pinned blocks are multiples of this
constexpr size_t kMinPinned = (size_t)1 << 20;   // below this, heap memory
constexpr size_t kIdleCap = (size_t)8 << 30;     // idle pinned bytes kept for reuse
constexpr size_t kLiveCap = (size_t)32 << 30;    // pinned bytes held by live results

// the public struct comes first, so a qp_result* is a Box*
struct Box {
    qp_result pub;
    void* block;
    size_t bytes;
    bool pinned;
};

class PinnedPool {
public:
    // a block of at least `want` bytes (rounded up to kGrain) or nullptr
    void* get(size_t want, size_t* got) {
        want = (want + kGrain - 1) / kGrain * kGrain;
        {
            std::lock_guard<std::mutex> g(mu_);
            // best fit among idle blocks, at most twice the size asked for
            auto it = idle_.lower_bound(want);
            if (it != idle_.end() && it->first <= 2 * want) {
                void* p = it->second;
                *got = it->first;
                idle_bytes_ -= it->first;
                live_bytes_ += it->first;
                idle_.erase(it);
                return p;
            }
            if (live_bytes_ + want > kLiveCap) return nullptr;
            live_bytes_ += want;  // reserved before the (slow) pinning call
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess || !p) {
            (void)hipGetLastError();
            std::lock_guard<std::mutex> g(mu_);
            live_bytes_ -= want;
            return nullptr;
        }
        *got = want;
        return p;
    }

    void put(void* p, size_t bytes) {
        {
            std::lock_guard<std::mutex> g(mu_);
            live_bytes_ -= bytes;
            if (idle_bytes_ + bytes <= kIdleCap) {
                idle_.emplace(bytes, p);
                idle_bytes_ += bytes;
                return;
            }
        }
        (void)hipHostFree(p);
    }

private:
    std::mutex mu_;
    std::multimap<size_t, void*> idle_;
    size_t idle_bytes_ = 0;
    size_t live_bytes_ = 0;
};

// never destroyed: results may be freed while the process exits
PinnedPool& pool() {
    static PinnedPool* p = new PinnedPool;
    return *p;
}

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

}  // namespace

qp_result* qp::result_alloc(int32_t n_seqs, int64_t P, int64_t rows, int64_t nnz) {
    if (P < 0 || rows < 0 || nnz < 0) return nullptr;
    const size_t p1 = (size_t)P + 1;
    // every array has at least one element, so no pointer is null
    const size_t sz[9] = {
        sizeof(int32_t) * std::max<size_t>(P, 1),        // pair_i
        sizeof(int32_t) * std::max<size_t>(P, 1),        // pair_j
        sizeof(int64_t) * p1,                            // row_off
        sizeof(int32_t) * std::max<size_t>(rows, 1),     // row_ptr
        sizeof(int64_t) * p1,                            // nnz_off
        sizeof(int32_t) * std::max<size_t>(nnz, 1),      // col
        sizeof(float) * std::max<size_t>(nnz, 1),        // val
        sizeof(double) * std::max<size_t>(P, 1),         // dist
        sizeof(double) * 2 * std::max<size_t>(P, 1),     // log_z
    };
    size_t total = 0;
    for (size_t s : sz) total += up(s);
    Box* b = static_cast<Box*>(std::calloc(1, sizeof(Box)));
    if (!b) return nullptr;
    size_t got = 0;
    void* blk = total >= kMinPinned ? pool().get(total, &got) : nullptr;
    if (blk) {
        b->pinned = true;
        b->bytes = got;
    } else {
        blk = std::aligned_alloc(kAlign, up(total));
        if (!blk) {
            std::free(b);
            return nullptr;
        }
        b->bytes = up(total);
    }
    b->block = blk;
    char* c = static_cast<char*>(blk);
    void* at[9];
    for (int k = 0; k < 9; ++k) {
        at[k] = c;
        c += up(sz[k]);
    }
    qp_result* r = &b->pub;
    r->n_seqs = n_seqs;
    r->n_pairs = P;
    r->total_rows = rows;
    r->nnz = nnz;
    r->pair_i = static_cast<int32_t*>(at[0]);
    r->pair_j = static_cast<int32_t*>(at[1]);
    r->row_off = static_cast<int64_t*>(at[2]);
    r->row_ptr = static_cast<int32_t*>(at[3]);
    r->nnz_off = static_cast<int64_t*>(at[4]);
    r->col = static_cast<int32_t*>(at[5]);
    r->val = static_cast<float*>(at[6]);
    r->dist = static_cast<double*>(at[7]);
    r->log_z = static_cast<double*>(at[8]);
    r->row_off[0] = 0;
    r->nnz_off[0] = 0;
    return r;
}

bool qp::result_pinned(const qp_result* r) { return r && reinterpret_cast<const Box*>(r)->pinned; }

extern "C" void qp_result_free(qp_result* r) {
    if (!r) return;
    Box* b = reinterpret_cast<Box*>(r);
    if (b->pinned)
        pool().put(b->block, b->bytes);
    else
        std::free(b->block);
    std::free(b);
}
