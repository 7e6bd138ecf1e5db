// Selective consistency on the device: every pair's sparse posterior matrix
// is relaxed through the third sequences the guide tree selects (paper:
// Methods, "Selective consistency"; "Other algorithmic improvements" for the
// number of passes).  For pair (x, y) with Z_xy = { z : max(d_xz, d_yz) <= T }
// (tree-guided distances) and h_xy = 1 + (h - 1) |Z_xy| / (k - 2):
//   S'_xy = (2 h_xy S_xy + sum_{z in Z_xy} S_xz S_zy) / (2 h_xy + |Z_xy|),
// entries below the sparsity threshold dropped; S_ab for a > b is S_ba
// transposed.  The paper names the transformation, its selection rule, the
// amplification and the pass count; the formula is the consistency
// transformation of the aligners the method descends from, read as above.
//
// Layout: the all-pairs CSR of the posterior stage (qp_device_result).  Once
// per run the pairs are ordered by their work (selected third sequences
// times rows), costliest first.  Per pass: (1) every pair's matrix is
// transposed into a CSR of the same entry range (rows = residues of the
// second sequence), so both orientations of every S_ab are rows of some CSR;
// (2) wavefronts take pairs in that order from a counter, one at a time, and
// accumulate each block of output rows in LDS -- lanes take (row, z) items,
// walk row i of S_xz eight entries at a time and, for each entry (k, v), row
// k of S_zy, adding v * S_zy(k, j) with LDS atomics -- then scale, threshold
// and compact each row in column order; (3) per-pair counts are scanned and
// the entries gathered in pair order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qp.h"
#include "qp_internal.h"
#include "qp_wave.h"

namespace {

using qp::kWave;
constexpr int kRelaxWaves = 4;       // wavefronts per block
constexpr int kMaxRelaxSeqs = 2048;  // a selected sequence is an int16 in the LDS list
constexpr int kRelaxGroup = 8;          // S_xz entries of one row taken together
constexpr int kQueueSlot = 8;           // flags[8 + pass]: the pair counter of each pass (at most 8 passes)
constexpr int kOrderBins = 64;          // cost bins of the pair order (costliest first)
constexpr int64_t kRelaxLds = 64 * 1024;  // dynamic LDS of a k_relax block

struct Csr {
    const int64_t* row_off;  // [P + 1] into row_ptr
    const int32_t* row_ptr;  // per pair: rows + 1 local pointers
    const int64_t* nnz_off;  // [P + 1] into col / val
    const int32_t* col;
    const float* val;
};

__device__ __forceinline__ int64_t pidx(int64_t a, int64_t b, int64_t k) { return a * k - a * (a + 1) / 2 + (b - a - 1); }

// transposes of every pair's matrix; the transposed rows of pair p are the
// columns of its second sequence, its entries occupy the same range of
// tr_col / tr_val as the pair's own, rows ascending within a column
__global__ __launch_bounds__(kWave * kRelaxWaves) void k_transpose(
    int32_t k, int64_t P, const int32_t* __restrict__ lens, const int32_t* __restrict__ pair_i,
    const int32_t* __restrict__ pair_j, Csr in, const int64_t* __restrict__ tr_row_off,
    int32_t* __restrict__ tr_row_ptr, int32_t* __restrict__ tr_col, float* __restrict__ tr_val,
    int* __restrict__ flags) {
    __shared__ int cnt_s[kRelaxWaves][qp::kMaxSeqLen + 1];
    __shared__ int rp_s[kRelaxWaves][qp::kMaxSeqLen + 1];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int* cnt = cnt_s[w];
    int* rp = rp_s[w];
    for (int64_t p = (int64_t)blockIdx.x * kRelaxWaves + w; p < P; p += (int64_t)gridDim.x * kRelaxWaves) {
        const int a = __builtin_amdgcn_readfirstlane(pair_i[p]);
        const int b = __builtin_amdgcn_readfirstlane(pair_j[p]);
        const int m = lens[a], n = lens[b];
        const int64_t base = in.nnz_off[p];
        const int ne = (int)(in.nnz_off[p + 1] - base);
        const int32_t* rpi = in.row_ptr + in.row_off[p];
        int32_t* rpo = tr_row_ptr + tr_row_off[p];
        for (int c = lane; c <= n; c += kWave) cnt[c] = 0;
        // an entry whose column lies outside the second sequence is left out
        // (and reported), so that nothing is written outside the pair's range
        for (int e0 = 0; e0 < ne; e0 += kWave) {
            const int e = e0 + lane;
            const int j = e < ne ? in.col[base + e] : 0;
            const bool valid = e < ne && j >= 0 && j < n;
            if (e < ne && !valid) atomicOr(flags, 4);
            qp::wave_count_add(cnt, valid ? j : 0, valid);
        }
        int carry = 0;
        for (int c0 = 0; c0 <= n; c0 += kWave) {
            const int c = c0 + lane;
            const int v = c < n ? cnt[c] : 0;
            const int inc = qp::wave_incl_scan(v, lane);
            if (c <= n) {
                rp[c] = carry + inc - v;
                rpo[c] = carry + inc - v;
            }
            carry += __shfl(inc, kWave - 1, kWave);
        }
        for (int c = lane; c <= n; c += kWave) cnt[c] = 0;
        for (int e0 = 0; e0 < ne; e0 += kWave) {
            const int e = e0 + lane;
            const int jr = e < ne ? in.col[base + e] : 0;
            const bool valid = e < ne && jr >= 0 && jr < n;
            const int j = valid ? jr : 0;
            // row of entry e: the last i with rpi[i] <= e (rpi[0] = 0, rpi[m] = ne)
            int lo = 0, hi = m;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rpi[mid] <= e) lo = mid;
                else hi = mid;
            }
            // entries are met in row order, so ranks within a column ascend with the row
            const int rank = qp::wave_count_add(cnt, j, valid);
            if (valid) {
                tr_col[base + rp[j] + rank] = lo;
                tr_val[base + rp[j] + rank] = in.val[base + e];
            }
        }
    }
}

// one pass of the relaxation; out_* receive per-pair row pointers and the
// kept entries at the pair's bound offset (stage_off), out_nnz the count.
// A wavefront relaxes its pair a block of B rows at a time: the selected
// third sequences are compacted once into an LDS list, the block's rows get
// B accumulator rows of acc_stride floats in LDS, and the (row, z) items of
// the block are dealt over the lanes, so every lane follows its own chain of
// dependent loads (row i of S_xz, then the rows of S_zy it points to) and the
// chains of the block overlap instead of running one row after another.
__global__ __launch_bounds__(kWave * kRelaxWaves) void k_relax(
    int32_t k, int64_t P, const int32_t* __restrict__ lens, const int32_t* __restrict__ pair_i,
    const int32_t* __restrict__ pair_j, Csr in, const int64_t* __restrict__ tr_row_off,
    const int32_t* __restrict__ tr_row_ptr, const int32_t* __restrict__ tr_col, const float* __restrict__ tr_val,
    const int32_t* __restrict__ tdist, int32_t T, float h, float thresh, int32_t cap,
    const int64_t* __restrict__ out_row_off, int32_t* __restrict__ out_row_ptr, const int64_t* __restrict__ stage_off,
    int32_t* __restrict__ stage_col, float* __restrict__ stage_val, int64_t* __restrict__ out_nnz,
    int* __restrict__ flags, int* __restrict__ queue, const int32_t* __restrict__ order, int32_t B,
    int32_t acc_stride) {
    // dynamic LDS: [kRelaxWaves][B][acc_stride] accumulators, then
    // [kRelaxWaves][k] selected third sequences
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    float* acc = lds + (int64_t)w * B * acc_stride;
    int16_t* zl = reinterpret_cast<int16_t*>(lds + (int64_t)kRelaxWaves * B * acc_stride) + (int64_t)w * k;
    // each wavefront takes the next pair of the cost order from the pass's
    // counter (zero at the start of the run) until none is left: the number
    // of third sequences, and so a pair's work, varies widely from pair to
    // pair.  Every lane
    // takes part in the atomic (lane 0 adds one, the others nothing), so no
    // branch on the lane index comes before the wave-wide read of its result
    // that the compiler could route some lanes around.
    for (;;) {
        const int q = __builtin_amdgcn_readfirstlane(atomicAdd(queue, lane == 0 ? 1 : 0));
        if (q >= P) break;
        const int64_t p = __builtin_amdgcn_readfirstlane(order[q]);
        const int x = __builtin_amdgcn_readfirstlane(pair_i[p]);
        const int y = __builtin_amdgcn_readfirstlane(pair_j[p]);
        const int m = lens[x], n = lens[y];
        // selection, compacted in increasing z
        int nsel = 0;
        for (int c = 0; c * kWave < k; ++c) {
            const int z = c * kWave + lane;
            bool s = z < k && z != x && z != y;
            if (s) {
                const int dxz = tdist[pidx(min(x, z), max(x, z), k)];
                const int dyz = tdist[pidx(min(y, z), max(y, z), k)];
                s = max(dxz, dyz) <= T;
            }
            const unsigned long long sm = __ballot(s);
            if (s) {
                const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(sm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sm, 0));
                zl[nsel + rank] = (int16_t)z;
            }
            nsel += __popcll(sm);
        }
        const float hxy = k <= 2 ? 1.f : 1.f + (h - 1.f) * (float)nsel / (float)(k - 2);
        const float own = 2.f * hxy;
        const float invW = 1.f / (2.f * hxy + (float)nsel);
        const int64_t bxy = in.nnz_off[p];
        const int32_t* rxy = in.row_ptr + in.row_off[p];
        int32_t* orp = out_row_ptr + out_row_off[p];
        const int64_t obase = stage_off[p];
        int count = 0;
        for (int i0 = 0; i0 < m; i0 += B) {
            const int nb = min(B, m - i0);
            for (int c = lane; c < nb * acc_stride; c += kWave) acc[c] = 0.f;
            // the pair's own entries, amplified (rows i0 .. i0+nb-1 are one
            // contiguous run of its CSR)
            const int e_lo = rxy[i0], e_hi = rxy[i0 + nb];
            for (int e = e_lo + lane; e < e_hi; e += kWave) {
                int r = 0;
                while (r + 1 < nb && rxy[i0 + r + 1] <= e) ++r;
                const int j = in.col[bxy + e];
                if (j >= 0 && j < n) acc[r * acc_stride + j] = own * in.val[bxy + e];
            }
            // (row, z) items of the block over the lanes, z-major: lanes next
            // to each other take the block's consecutive rows of one S_xz, whose
            // row pointers and entries share cache lines, and whose entries point
            // to neighbouring rows of S_zy
            const int items = nb * nsel;
            for (int q = lane; q < items; q += kWave) {
                const int zi = q / nb;
                const int r = q - zi * nb;
                const int z = zl[zi];
                const int i = i0 + r;
                // row i of S_xz: pair (x, z) as stored, or (z, x) transposed
                const bool xa = x < z;
                const int64_t pxz = xa ? pidx(x, z, k) : pidx(z, x, k);
                const int32_t* ra = xa ? in.row_ptr + in.row_off[pxz] : tr_row_ptr + tr_row_off[pxz];
                const int32_t* ca = xa ? in.col : tr_col;
                const float* va = xa ? in.val : tr_val;
                const int64_t ba = in.nnz_off[pxz];
                // rows of S_zy: pair (z, y) as stored, or (y, z) transposed
                const bool za = z < y;
                const int64_t pzy = za ? pidx(z, y, k) : pidx(y, z, k);
                const int32_t* rb = za ? in.row_ptr + in.row_off[pzy] : tr_row_ptr + tr_row_off[pzy];
                const int32_t* cb = za ? in.col : tr_col;
                const float* vb = za ? in.val : tr_val;
                const int64_t bb = in.nnz_off[pzy];
                float* accr = acc + r * acc_stride;
                const int ea1 = ra[i + 1];
                // up to kRelaxGroup entries of row i at a time: their columns,
                // then the row ranges of S_zy they select, then those rows
                // walked side by side, so each round has a group's loads in
                // flight instead of one chain of dependent loads per entry
                for (int eg = ra[i]; eg < ea1; eg += kRelaxGroup) {
                    int kk[kRelaxGroup], lo[kRelaxGroup], len[kRelaxGroup];
                    float v1[kRelaxGroup];
#pragma unroll
                    for (int u = 0; u < kRelaxGroup; ++u) {
                        const int e = eg + u < ea1 ? eg + u : eg;  // a stored entry either way
                        kk[u] = ca[ba + e];
                        v1[u] = va[ba + e];
                    }
                    int rounds = 0;
#pragma unroll
                    for (int u = 0; u < kRelaxGroup; ++u) {
                        lo[u] = rb[kk[u]];
                        len[u] = eg + u < ea1 ? rb[kk[u] + 1] - lo[u] : 0;
                        rounds = max(rounds, len[u]);
                    }
                    for (int t = 0; t < rounds; ++t) {
                        int jj[kRelaxGroup];
                        float ww[kRelaxGroup];
#pragma unroll
                        for (int u = 0; u < kRelaxGroup; ++u) {
                            const bool ok = t < len[u];
                            // past its row: entry eg of S_xz, stored in every entry array
                            const int64_t eb = ok ? bb + lo[u] + t : ba + eg;
                            jj[u] = ok ? cb[eb] : -1;
                            ww[u] = vb[eb];
                        }
#pragma unroll
                        for (int u = 0; u < kRelaxGroup; ++u)
                            if (jj[u] >= 0 && jj[u] < n) atomicAdd(&accr[jj[u]], v1[u] * ww[u]);
                    }
                }
            }
            // scale, threshold, compact each row in column order (at most cap)
            for (int r = 0; r < nb; ++r) {
                const float* accr = acc + r * acc_stride;
                int rc = 0;
                for (int c0 = 0; c0 < n; c0 += kWave) {
                    const int c = c0 + lane;
                    const float v = c < n ? accr[c] * invW : 0.f;
                    const bool hit = c < n && v >= thresh;
                    const unsigned long long hm = __ballot(hit);
                    const int rank = rc + __popcll(hm & (lane == 0 ? 0ull : (~0ull >> (kWave - lane))));
                    if (hit && rank < cap) {
                        stage_col[obase + count + rank] = c;
                        stage_val[obase + count + rank] = v;
                    }
                    rc += __popcll(hm);
                }
                if (rc > cap) {
                    if (lane == 0) atomicOr(flags, 2);
                    rc = cap;
                }
                count += rc;
                if (lane == 0) orp[i0 + r + 1] = count;
            }
        }
        if (lane == 0) {
            orp[0] = 0;
            out_nnz[p] = count;
        }
    }
}

// The order in which the wavefronts take pairs: by the pair's work, about
// its selected third sequences times its rows, in bins a third of an octave
// wide, the costliest bin first (pairs with nothing selected last), so that
// no expensive pair starts when the others are nearly done.  bins holds
// [kOrderBins] counts, [kOrderBins] first slots, [kOrderBins] fill counters.
__global__ void k_order_keys(int32_t k, int64_t P, const int32_t* __restrict__ lens,
                             const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
                             const int32_t* __restrict__ tdist, int32_t T, int32_t* __restrict__ key,
                             int* __restrict__ bins) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int x = pair_i[p], y = pair_j[p];
    int nsel = 0;
    for (int z = 0; z < k; ++z) {
        if (z == x || z == y) continue;
        const int dxz = tdist[pidx(min(x, z), max(x, z), k)];
        const int dyz = tdist[pidx(min(y, z), max(y, z), k)];
        nsel += max(dxz, dyz) <= T ? 1 : 0;
    }
    const float cost = (float)nsel * (float)lens[x];
    const int kb = nsel == 0 ? 0 : min(kOrderBins - 1, 1 + (int)(3.f * log2f(cost)));
    key[p] = kb;
    atomicAdd(&bins[kb], 1);
}

__global__ void k_order_starts(int* __restrict__ bins) {
    if (threadIdx.x != 0) return;
    int at = 0;
    for (int b = kOrderBins - 1; b >= 0; --b) {
        bins[kOrderBins + b] = at;
        at += bins[b];
    }
}

__global__ void k_order_fill(int64_t P, const int32_t* __restrict__ key, int* __restrict__ bins,
                             int32_t* __restrict__ order) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int kb = key[p];
    order[bins[kOrderBins + kb] + atomicAdd(&bins[2 * kOrderBins + kb], 1)] = (int32_t)p;
}

__global__ void k_zero_i32(int* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace

struct qp_relax {
    int device = 0;
    int32_t k = 0;
    int64_t P = 0;
    int32_t T = 0;
    double h = 1.0;
    int32_t passes = 1;
    float thresh = 0.f;
    int32_t cap = 1;
    int n_cu = 1;
    int32_t rows_per_block = 1;  // rows a wavefront relaxes at once (B)
    int32_t acc_stride = 1;      // LDS accumulator row (>= the longest second sequence)
    int64_t lds_bytes = 0;       // dynamic LDS of a k_relax block
    std::vector<int32_t> lens;
    int64_t total_rows = 0, tr_rows = 0, bound = 0, in_cap = 0;
    std::vector<void*> allocs;
    int32_t *d_lens = nullptr, *d_pi = nullptr, *d_pj = nullptr;
    int64_t *d_row_off = nullptr, *d_tr_row_off = nullptr, *d_stage_off = nullptr;
    int32_t* d_tr_row_ptr = nullptr;
    int32_t* d_tr_col = nullptr;
    float* d_tr_val = nullptr;
    int32_t* d_stage_col = nullptr;
    float* d_stage_val = nullptr;
    // two output sets: pass q writes set q % 2
    int32_t* d_out_row_ptr[2] = {};
    int64_t* d_out_nnz[2] = {};
    int32_t* d_out_col[2] = {};
    float* d_out_val[2] = {};
    int64_t* d_scan_tmp = nullptr;
    int* d_flags = nullptr;
    int32_t* d_key = nullptr;    // [P] cost bin of each pair
    int32_t* d_order = nullptr;  // [P] pairs, costliest first
    int* d_bins = nullptr;       // [3 * kOrderBins] counts, first slots, fill counters
    hipStream_t last_stream = nullptr;
    hipEvent_t done = nullptr;
    bool ran = false;
    int last_set = 0;
    int64_t last_nnz = 0;
};

namespace {

qp_status relax_alloc(qp_relax* r, void** p, int64_t bytes) {
    bytes = std::max<int64_t>(bytes, 4);
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return qp::fail_msg(QP_ENOMEM, "hipMalloc of %lld bytes for the relaxation failed: %s", (long long)bytes,
                            hipGetErrorString(e));
    }
    r->allocs.push_back(*p);
    return QP_OK;
}

void relax_free(qp_relax* r) {
    if (r->ran && r->done) hipEventSynchronize(r->done);
    for (void* p : r->allocs) hipFree(p);
    r->allocs.clear();
    if (r->done) hipEventDestroy(r->done);
    r->done = nullptr;
}

#define RX_TRY(expr)                                                                                       \
    do {                                                                                                   \
        hipError_t _e = (expr);                                                                            \
        if (_e != hipSuccess) return qp::fail_msg(QP_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

}  // namespace

extern "C" {

qp_status qp_relax_create(const int32_t* lens, int32_t n, int64_t in_capacity, int32_t tree_threshold,
                          double amplification, int32_t passes, float thresh, qp_relax** out) {
    if (!out) return qp::fail_msg(QP_EINVAL, "out is NULL");
    *out = nullptr;
    qp_status st = qp::validate_lens(lens, n);
    if (st != QP_OK) return st;
    if (n > kMaxRelaxSeqs) return qp::fail_msg(QP_EINVAL, "n = %d sequences: at most %d", n, kMaxRelaxSeqs);
    if (tree_threshold < 0) return qp::fail_msg(QP_EINVAL, "tree_threshold = %d < 0", tree_threshold);
    if (!(amplification >= 1.0) || !std::isfinite(amplification))
        return qp::fail_msg(QP_EINVAL, "amplification = %g is not >= 1", amplification);
    if (passes < 1 || passes > 8) return qp::fail_msg(QP_EINVAL, "passes = %d is not in [1, 8]", passes);
    if (!(thresh > 0.0f && thresh <= 1.0f)) return qp::fail_msg(QP_EINVAL, "thresh = %g is not in (0, 1]", (double)thresh);
    if (in_capacity < 0) return qp::fail_msg(QP_EINVAL, "in_capacity = %lld < 0", (long long)in_capacity);
    int dev = 0, n_cu = 0;
    if ((st = qp::check_device(&dev, &n_cu)) != QP_OK) return st;
    qp_relax* r = new (std::nothrow) qp_relax();
    if (!r) return qp::fail_msg(QP_ENOMEM, "out of host memory");
    r->device = dev;
    r->n_cu = n_cu;
    r->k = n;
    r->P = (int64_t)n * (n - 1) / 2;
    r->T = tree_threshold;
    r->h = amplification;
    r->passes = passes;
    r->thresh = thresh;
    r->cap = (int32_t)std::min<double>(qp::kMaxSeqLen, std::floor(1.0 / (double)thresh) + 1.0);
    r->lens.assign(lens, lens + n);
    {
        // B accumulator rows per wavefront, as many (up to 8) as fit beside
        // the selection lists in the LDS a block may hold: the more rows of
        // one S_xz neighbouring lanes take, the more their loads share lines
        const int32_t nmax = *std::max_element(lens, lens + n);
        r->acc_stride = nmax + (nmax & 1);
        const int64_t zl_bytes = (int64_t)kRelaxWaves * n * 2;
        const int64_t per_row = (int64_t)kRelaxWaves * r->acc_stride * 4;
        r->rows_per_block = (int32_t)std::max<int64_t>(1, std::min<int64_t>(8, (kRelaxLds - zl_bytes) / per_row));
        r->lds_bytes = (int64_t)r->rows_per_block * per_row + zl_bytes;
        if (r->lds_bytes > kRelaxLds) {
            delete r;
            return qp::fail_msg(QP_EINVAL, "the relaxation's LDS (%lld bytes) does not fit a block", (long long)r->lds_bytes);
        }
    }
    const int64_t P = r->P;
    std::vector<int32_t> pi((size_t)std::max<int64_t>(P, 1)), pj((size_t)std::max<int64_t>(P, 1));
    std::vector<int64_t> row_off((size_t)P + 1), tr_off((size_t)P + 1), stage_off((size_t)P + 1);
    {
        int64_t q = 0, ro = 0, to = 0, so = 0;
        for (int32_t i = 0; i + 1 < n; ++i)
            for (int32_t j = i + 1; j < n; ++j, ++q) {
                pi[q] = i;
                pj[q] = j;
                row_off[q] = ro;
                tr_off[q] = to;
                stage_off[q] = so;
                ro += lens[i] + 1;
                to += lens[j] + 1;
                so += (int64_t)lens[i] * qp::row_bound(lens[j], thresh);
            }
        row_off[P] = ro;
        tr_off[P] = to;
        stage_off[P] = so;
        r->total_rows = ro;
        r->tr_rows = to;
        r->bound = std::max<int64_t>(so, 1);
    }
    // the input holds at most its own bound; a caller may give the exact count
    r->in_cap = in_capacity > 0 ? in_capacity : r->bound;
    qp_status as = QP_OK;
    auto A = [&](void** p, int64_t b) {
        if (as == QP_OK) as = relax_alloc(r, p, b);
    };
    A((void**)&r->d_lens, 4LL * n);
    A((void**)&r->d_pi, 4 * P);
    A((void**)&r->d_pj, 4 * P);
    A((void**)&r->d_row_off, 8 * (P + 1));
    A((void**)&r->d_tr_row_off, 8 * (P + 1));
    A((void**)&r->d_stage_off, 8 * (P + 1));
    A((void**)&r->d_tr_row_ptr, 4 * r->tr_rows);
    // transposed copies hold the input of a pass: the caller's first input,
    // then (second pass on) a relaxed output, which stays within the bound
    const int64_t tr_cap = passes > 1 ? std::max(r->in_cap, r->bound) : r->in_cap;
    A((void**)&r->d_tr_col, 4 * tr_cap);
    A((void**)&r->d_tr_val, 4 * tr_cap);
    A((void**)&r->d_stage_col, 4 * r->bound);
    A((void**)&r->d_stage_val, 4 * r->bound);
    for (int q = 0; q < (passes > 1 ? 2 : 1); ++q) {
        A((void**)&r->d_out_row_ptr[q], 4 * r->total_rows);
        A((void**)&r->d_out_nnz[q], 8 * (P + 1));
        A((void**)&r->d_out_col[q], 4 * r->bound);
        A((void**)&r->d_out_val[q], 4 * r->bound);
    }
    A((void**)&r->d_scan_tmp, 8 * (qp::scan_tmp_elems(P + 1) + 8));
    A((void**)&r->d_flags, 64);
    A((void**)&r->d_key, 4 * P);
    A((void**)&r->d_order, 4 * P);
    A((void**)&r->d_bins, 4 * 3 * kOrderBins);
    if (as != QP_OK) {
        relax_free(r);
        delete r;
        return as;
    }
    hipError_t e = hipMemcpy(r->d_lens, lens, 4ull * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && P > 0) e = hipMemcpy(r->d_pi, pi.data(), 4ull * P, hipMemcpyHostToDevice);
    if (e == hipSuccess && P > 0) e = hipMemcpy(r->d_pj, pj.data(), 4ull * P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_row_off, row_off.data(), 8ull * (P + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_tr_row_off, tr_off.data(), 8ull * (P + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_stage_off, stage_off.data(), 8ull * (P + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        relax_free(r);
        delete r;
        return qp::fail_msg(QP_EDEVICE, "relaxation set-up failed: %s", hipGetErrorString(e));
    }
    *out = r;
    return QP_OK;
}

qp_status qp_relax_run(qp_relax* r, const qp_device_result* in, int64_t in_nnz, const int32_t* d_tdist,
                       void* stream) {
    if (!r) return qp::fail_msg(QP_EINVAL, "relax is NULL");
    if (!in) return qp::fail_msg(QP_EINVAL, "in is NULL");
    if (in->n_pairs != r->P)
        return qp::fail_msg(QP_EINVAL, "input holds %lld pairs, the family %lld", (long long)in->n_pairs,
                            (long long)r->P);
    if (in->total_rows != r->total_rows)
        return qp::fail_msg(QP_EINVAL, "input holds %lld row pointers, the family %lld", (long long)in->total_rows,
                            (long long)r->total_rows);
    if (in_nnz < 0 || in_nnz > r->in_cap)
        return qp::fail_msg(QP_EINVAL, "input holds %lld entries, more than the %lld this relaxation was made for",
                            (long long)in_nnz, (long long)r->in_cap);
    if (r->P > 0 && (!in->row_off || !in->row_ptr || !in->nnz_off || !in->col || !in->val || !d_tdist))
        return qp::fail_msg(QP_EINVAL, "a device input array is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    RX_TRY(hipSetDevice(r->device));
    if (r->ran) RX_TRY(hipEventSynchronize(r->done));  // one run at a time per relaxation
    r->last_stream = s;
    r->ran = true;
    r->last_set = 0;
    if (r->P == 0) {
        RX_TRY(hipEventRecord(r->done, s));
        return QP_OK;
    }
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, r->d_flags, 16);
    RX_TRY(hipGetLastError());
    {
        const unsigned og = (unsigned)((r->P + 255) / 256);
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, r->d_bins, 3 * kOrderBins);
        RX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_order_keys, dim3(og), dim3(256), 0, s, r->k, r->P, r->d_lens, r->d_pi, r->d_pj,
                           d_tdist, r->T, r->d_key, r->d_bins);
        RX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_order_starts, dim3(1), dim3(64), 0, s, r->d_bins);
        RX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_order_fill, dim3(og), dim3(256), 0, s, r->P, r->d_key, r->d_bins, r->d_order);
        RX_TRY(hipGetLastError());
    }
    const int64_t waves_wanted = (r->P + kRelaxWaves - 1) / kRelaxWaves;
    const unsigned grid = (unsigned)std::min<int64_t>(waves_wanted, (int64_t)r->n_cu * 8);
    Csr cur{in->row_off, in->row_ptr, in->nnz_off, in->col, in->val};
    for (int pass = 0; pass < r->passes; ++pass) {
        const int q = pass & 1;
        hipLaunchKernelGGL(k_transpose, dim3(grid), dim3(kWave * kRelaxWaves), 0, s, r->k, r->P, r->d_lens, r->d_pi,
                           r->d_pj, cur, r->d_tr_row_off, r->d_tr_row_ptr, r->d_tr_col, r->d_tr_val, r->d_flags);
        RX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_relax, dim3(grid), dim3(kWave * kRelaxWaves), (size_t)r->lds_bytes, s, r->k, r->P,
                           r->d_lens, r->d_pi, r->d_pj, cur, r->d_tr_row_off, r->d_tr_row_ptr, r->d_tr_col,
                           r->d_tr_val, d_tdist, r->T, (float)r->h, r->thresh, r->cap, r->d_row_off,
                           r->d_out_row_ptr[q], r->d_stage_off, r->d_stage_col, r->d_stage_val, r->d_out_nnz[q],
                           r->d_flags, r->d_flags + kQueueSlot + pass, r->d_order, r->rows_per_block,
                           r->acc_stride);
        RX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(r->d_out_nnz[q] + r->P), 2);
        RX_TRY(hipGetLastError());
        RX_TRY(qp::scan_i64(r->d_out_nnz[q], r->P + 1, r->d_scan_tmp, s));
        RX_TRY(qp::launch_gather(r->P, r->d_out_nnz[q], r->d_stage_off, r->d_stage_col, r->d_stage_val,
                                 r->d_out_col[q], r->d_out_val[q], r->bound, s));
        cur = Csr{r->d_row_off, r->d_out_row_ptr[q], r->d_out_nnz[q], r->d_out_col[q], r->d_out_val[q]};
        r->last_set = q;
    }
    RX_TRY(hipEventRecord(r->done, s));
    return QP_OK;
}

qp_status qp_relax_sync(qp_relax* r, qp_device_result* out) {
    if (!r) return qp::fail_msg(QP_EINVAL, "relax is NULL");
    if (!r->ran) return qp::fail_msg(QP_EINVAL, "relaxation has not been run");
    RX_TRY(hipSetDevice(r->device));
    RX_TRY(hipEventSynchronize(r->done));
    int64_t nnz = 0;
    int flags = 0;
    if (r->P > 0) {
        RX_TRY(hipMemcpy(&nnz, r->d_out_nnz[r->last_set] + r->P, 8, hipMemcpyDeviceToHost));
        RX_TRY(hipMemcpy(&flags, r->d_flags, 4, hipMemcpyDeviceToHost));
    }
    r->last_nnz = nnz;
    if (flags & 4) return qp::fail_msg(QP_EINVAL, "an input entry's column lies outside its pair's second sequence");
    if (flags & 2) return qp::fail_msg(QP_EDEVICE, "a relaxed row held more entries than its slots");
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->n_pairs = r->P;
        out->total_rows = r->total_rows;
        out->nnz = nnz;
        out->pair_i = r->d_pi;
        out->pair_j = r->d_pj;
        out->row_off = r->d_row_off;
        out->row_ptr = r->d_out_row_ptr[r->last_set];
        out->nnz_off = r->d_out_nnz[r->last_set];
        out->col = r->d_out_col[r->last_set];
        out->val = r->d_out_val[r->last_set];
    }
    return QP_OK;
}

qp_status qp_relax_download(qp_relax* r, qp_result** out) {
    if (!out) return qp::fail_msg(QP_EINVAL, "out is NULL");
    *out = nullptr;
    qp_device_result d;
    qp_status st = qp_relax_sync(r, &d);
    if (st != QP_OK) return st;
    qp_result* res = qp::result_alloc(r->k, r->P, r->total_rows, d.nnz);
    if (!res) return qp::fail_msg(QP_ENOMEM, "out of host memory");
    res->thresh = r->thresh;
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t b) {
        if (e == hipSuccess && b) e = hipMemcpy(dst, src, b, hipMemcpyDeviceToHost);
    };
    if (r->P > 0) {
        cp(res->pair_i, d.pair_i, 4 * r->P);
        cp(res->pair_j, d.pair_j, 4 * r->P);
        cp(res->row_off, d.row_off, 8 * (r->P + 1));
        cp(res->row_ptr, d.row_ptr, 4 * r->total_rows);
        cp(res->nnz_off, d.nnz_off, 8 * (r->P + 1));
        cp(res->col, d.col, 4 * d.nnz);
        cp(res->val, d.val, 4 * d.nnz);
    }
    if (e != hipSuccess) {
        qp_result_free(res);
        return qp::fail_msg(QP_EDEVICE, "device-to-host copy failed: %s", hipGetErrorString(e));
    }
    *out = res;
    return QP_OK;
}

int64_t qp_relax_device_bytes(const qp_relax* r) {
    if (!r) return 0;
    int64_t b = 0;
    const int64_t P = r->P;
    const int64_t tr_cap = r->passes > 1 ? std::max(r->in_cap, r->bound) : r->in_cap;
    b += 4 * (int64_t)r->k + 8 * P + 24 * (P + 1) + 4 * r->tr_rows + 8 * tr_cap + 8 * r->bound;
    b += 8 * P + 4 * 3 * kOrderBins;  // the pair order
    b += (r->passes > 1 ? 2 : 1) * (4 * r->total_rows + 8 * (P + 1) + 8 * r->bound);
    return b;
}

void qp_relax_destroy(qp_relax* r) {
    if (!r) return;
    hipSetDevice(r->device);
    relax_free(r);
    delete r;
}

}  // extern "C"
