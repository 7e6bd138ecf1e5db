// Allocation-free entry point (qp_posteriors_noalloc): the device-resident
// pipeline of a plan sized to the output bound, with every workspace buffer
// carved out of one fixed device array instead of device allocations, and
// every step launched directly on the caller's stream.  For callers that
// cannot allocate: code under stream capture, tight serving loops, harnesses
// that forbid device allocation.  See include/qp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "qp.h"
#include "qp_internal.h"

namespace {

// The workspace.  Each device the library runs on holds its own copy until
// the process ends.  Its name is a host-side stand-in in host code: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[QP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
int g_cu[kMaxDevices] = {};

// layout of the counters at the start of the workspace (ints)
constexpr int kIntHeads = 0;                       // [kClasses] queue heads
constexpr int kIntFlags = 12;                      // status bits
constexpr int kIntHist = 16;                       // [kKeyBins]
constexpr int kIntFill = kIntHist + qp::kKeyBins;  // [kKeyBins]
constexpr int kIntPool = kIntFill + qp::kKeyBins;  // 64-bit pool head (8-byte aligned)
constexpr int kNumInts = kIntPool + 2;
static_assert(kIntPool % 2 == 0, "the pool head is a 64-bit counter");

int64_t up256(int64_t b) { return (b + 255) & ~int64_t(255); }

// zero the counters and the status word; row_off[P] / nnz_off[P] are set by
// the setup kernel
__global__ void k_na_clear(int* __restrict__ ints, int n, int32_t* __restrict__ status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ints[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

// a block of up to kPutWords 32-bit words carried in the kernel arguments,
// written to dst (host data reaches the device without a copy from pageable
// memory or a staging allocation)
constexpr int kPutWords = 256;
struct PutBlock {
    uint32_t w[kPutWords];
};
__global__ void k_na_put(uint32_t* __restrict__ dst, int count, PutBlock b) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = b.w[i];
}

// padded length of every sequence (the aligned copy's slot), scanned later
__global__ void k_na_pad(const int32_t* __restrict__ lens, int32_t n, int64_t* __restrict__ off) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
        off[i] = i < n ? (int64_t)((lens[i] + 3) & ~3) : 0;
}

// the empty family: row_off[0] = nnz_off[0] = 0 and a clear status
__global__ void k_na_empty(int64_t* __restrict__ row_off, int64_t* __restrict__ nnz_off, int32_t* __restrict__ status) {
    if (threadIdx.x == 0) {
        row_off[0] = 0;
        nnz_off[0] = 0;
        *status = 0;
    }
}

// status word for the caller: the pipeline's flag bits
__global__ void k_na_status(const int* __restrict__ flags, int32_t* __restrict__ status) {
    if (threadIdx.x == 0) *status = *flags;
}

hipError_t put(uint32_t* dst, const void* src, size_t bytes, hipStream_t s) {
    const uint32_t* w = static_cast<const uint32_t*>(src);
    const size_t words = (bytes + 3) / 4;
    for (size_t at = 0; at < words; at += kPutWords) {
        PutBlock b;
        const int cnt = (int)std::min<size_t>(kPutWords, words - at);
        std::memset(&b, 0, sizeof(b));
        std::memcpy(b.w, w + at, std::min<size_t>((size_t)cnt * 4, bytes - at * 4));
        hipLaunchKernelGGL(k_na_put, dim3(1), dim3(256), 0, s, dst + at, cnt, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// the device address of this device's workspace, looked up once per device
// (with that device current) and kept
qp_status scratch_of(int dev, char** out, int* n_cu) {
    if (dev < 0 || dev >= kMaxDevices) return qp::fail_msg(QP_EDEVICE, "device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return qp::fail_msg(QP_EDEVICE, "hipGetSymbolAddress of the fixed workspace failed: %s", hipGetErrorString(e));
        }
        int cu = 0;
        e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || cu <= 0) {
            (void)hipGetLastError();
            return qp::fail_msg(QP_EDEVICE, "compute-unit count of device %d unavailable", dev);
        }
        g_ptr[dev] = p;
        g_cu[dev] = cu;
    }
    *out = static_cast<char*>(g_ptr[dev]);
    *n_cu = g_cu[dev];
    return QP_OK;
}

}  // namespace

#define NA_TRY(expr)                                                                                       \
    do {                                                                                                   \
        hipError_t _e = (expr);                                                                            \
        if (_e != hipSuccess) return qp::fail_msg(QP_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

extern "C" qp_status qp_posteriors_noalloc(const uint8_t* d_seqs, const int64_t* d_seq_off, const int32_t* lens,
                                           int32_t n, const qp_params* params, float thresh,
                                           const qp_noalloc_out* out, void* stream) {
    qp_status st = qp::validate_lens(lens, n);
    if (st != QP_OK) return st;
    if ((st = qp_params_check(params)) != QP_OK) return st;
    if (!(thresh > 0.0f && thresh <= 1.0f))
        return qp::fail_msg(QP_EINVAL, "thresh = %g is not in (0, 1]", (double)thresh);
    if (!out) return qp::fail_msg(QP_EINVAL, "out is NULL");
    if (!out->row_off || !out->nnz_off || !out->status)
        return qp::fail_msg(QP_EINVAL, "out->row_off, out->nnz_off and out->status are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t P = (int64_t)n * (n - 1) / 2;
    if (P > INT32_MAX) return qp::fail_msg(QP_EINVAL, "%lld pairs exceed the 2^31 limit", (long long)P);
    if (P == 0) {
        int dev = 0, n_cu = 0;
        char* ws = nullptr;
        if ((st = qp::check_device(&dev, nullptr)) != QP_OK) return st;
        if ((st = scratch_of(dev, &ws, &n_cu)) != QP_OK) return st;
        hipLaunchKernelGGL(k_na_empty, dim3(1), dim3(64), 0, s, out->row_off, out->nnz_off, out->status);
        NA_TRY(hipGetLastError());
        return QP_OK;
    }
    if (!d_seqs || !d_seq_off) return qp::fail_msg(QP_EINVAL, "device sequence pointers are NULL");
    if (!out->pair_i || !out->pair_j || !out->row_ptr || !out->col || !out->val || !out->dist || !out->log_z)
        return qp::fail_msg(QP_EINVAL, "an output array of qp_noalloc_out is NULL");

    // shape of the work per kernel class (as a plan sized to the bound)
    qp::ClassMap cmap{};
    double frac[qp::kClasses];
    int recompute[qp::kClasses];
    qp::current_tuning(&cmap, frac, recompute);
    struct Cls {
        int64_t pairs = 0;
        int mmax = 1, nmax = 1;
    } cls[qp::kClasses];
    int64_t rows = 0, bound = 0, seq_bytes = 0;
    int mmax = 1;
    for (int32_t i = 0; i < n; ++i) {
        mmax = std::max(mmax, lens[i]);
        seq_bytes += (lens[i] + 3) & ~3;
    }
    for (int32_t i = 0; i + 1 < n; ++i) {
        const int32_t m = lens[i];
        Cls& c = cls[qp::pair_class(m, cmap)];
        for (int32_t j = i + 1; j < n; ++j) {
            c.pairs += 1;
            c.mmax = std::max(c.mmax, m);
            c.nmax = std::max(c.nmax, lens[j]);
            rows += m + 1;
            bound += (int64_t)m * qp::row_bound(lens[j], thresh);
        }
    }
    bound = std::max<int64_t>(bound, 1);
    if (out->capacity < bound)
        return qp::fail_msg(QP_EINVAL, "out->capacity = %lld entries is below the output bound %lld (qp_output_bound)",
                            (long long)out->capacity, (long long)bound);
    int dev = 0;
    if ((st = qp::check_device(&dev, nullptr)) != QP_OK) return st;
    char* ws = nullptr;
    int n_cu = 0;
    if ((st = scratch_of(dev, &ws, &n_cu)) != QP_OK) return st;
    const int fp64 = params->precision == QP_FP64 ? 1 : 0;
    const double inv = std::floor(1.0 / (double)thresh);
    qp::PairArgs cargs[qp::kClasses];
    bool ck[qp::kClasses] = {};
    int64_t slot_max = 0;
    for (int c = 0; c < qp::kClasses; ++c) {
        if (!cls[c].pairs) continue;
        ck[c] = !fp64 && recompute[c] != 0;
        const int R = qp::class_rows(c, ck[c]);
        const int H = qp::kWave * R;
        const int nb = qp::class_banded(c) ? (cls[c].mmax + H - 1) / H : 1;
        const int cap = (int)std::max(1.0, std::min((double)cls[c].nmax, inv + 1.0));
        cargs[c] = qp::PairArgs{};
        qp::slot_layout(R, cls[c].mmax, cls[c].nmax, nb, cap, fp64, ck[c], &cargs[c]);
        cargs[c].cap = cap;
        slot_max = std::max(slot_max, cargs[c].slot_bytes);
    }

    // carve the workspace
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += up256(std::max<int64_t>(bytes, 1));
        return ws + at;
    };
    int* d_ints = reinterpret_cast<int*>(take((int64_t)kNumInts * 4));
    qp::DevParams* d_params = reinterpret_cast<qp::DevParams*>(take(sizeof(qp::DevParams)));
    void* d_tab = take((int64_t)qp::kTabRows * qp::kTabW * (fp64 ? 16 : 8));
    void* d_col0 = take((int64_t)mmax * (int64_t)qp::col0_bytes() + 64);
    qp::DevConsts* d_consts = reinterpret_cast<qp::DevConsts*>(take(sizeof(qp::DevConsts)));
    int32_t* d_lens = reinterpret_cast<int32_t*>(take((int64_t)n * 4));
    int64_t* d_seqa_off = reinterpret_cast<int64_t*>(take((int64_t)(n + 1) * 8));
    uint8_t* d_seqa = reinterpret_cast<uint8_t*>(take(seq_bytes + 4));
    int32_t* d_key = reinterpret_cast<int32_t*>(take(P * 4));
    int* d_bin_start = reinterpret_cast<int*>(take((int64_t)qp::kKeyBins * 4));
    int32_t* d_queue = reinterpret_cast<int32_t*>(take(P * 4));
    int64_t* d_base = reinterpret_cast<int64_t*>(take(P * 8));
    const int64_t scan_elems = std::max(qp::scan_tmp_elems(P + 1), qp::scan_tmp_elems((int64_t)n + 1)) + 8;
    int64_t* d_scan_tmp = reinterpret_cast<int64_t*>(take(scan_elems * 8));
    int32_t* d_pool_col = reinterpret_cast<int32_t*>(take(bound * 4));
    float* d_pool_val = reinterpret_cast<float*>(take(bound * 4));
    const int64_t fixed = off;
    const int64_t room = (int64_t)QP_NOALLOC_SCRATCH_BYTES - fixed;
    const int64_t slots = room > 0 ? room / slot_max : 0;
    if (slots < qp::kWavesPerBlock)
        return qp::fail_msg(QP_ENOMEM,
                            "the family needs %lld bytes of workspace for its tables, pair lists and an output pool "
                            "of %lld entries plus %lld bytes per wave for at least %d waves; the fixed workspace "
                            "holds %lld bytes (QP_NOALLOC_SCRATCH_BYTES)",
                            (long long)fixed, (long long)bound, (long long)slot_max, qp::kWavesPerBlock,
                            (long long)QP_NOALLOC_SCRATCH_BYTES);
    char* d_slots = ws + fixed;

    // the shared launch arguments
    qp::PairArgs a{};
    a.lens = d_lens;
    a.seqs = d_seqa;
    a.seq_off = d_seqa_off;
    a.pair_i = out->pair_i;
    a.pair_j = out->pair_j;
    a.queue = d_queue;
    a.n_pairs = P;
    a.queue_head = d_ints + kIntHeads;
    a.hist = d_ints + kIntHist;
    a.bin_start = d_bin_start;
    a.tab = d_tab;
    a.col0 = d_col0;
    a.consts = d_consts;
    a.thresh = thresh;
    a.cap_thresh = (int)std::min<double>(qp::kMaxSeqLen + 1, std::floor(1.0 / (double)thresh) + 1.0);
    a.row_off = out->row_off;
    a.row_ptr = out->row_ptr;
    a.pair_nnz = out->nnz_off;
    a.pair_base = d_base;
    a.pool_col = d_pool_col;
    a.pool_val = d_pool_val;
    a.pool_cap = bound;
    a.pool_head = reinterpret_cast<unsigned long long*>(d_ints + kIntPool);
    a.dist = out->dist;
    a.logz = out->log_z;
    a.flags = d_ints + kIntFlags;

    qp::DevParams dp{};
    std::memcpy(dp.joint, params->joint, sizeof(dp.joint));
    std::memcpy(dp.score, params->score, sizeof(dp.score));
    for (int k = 0; k < 2; ++k) {
        dp.gap_open[k] = k < params->n_gap_classes ? params->gap_open[k] : 0.0;
        dp.gap_extend[k] = k < params->n_gap_classes ? params->gap_extend[k] : 0.0;
    }
    dp.pf_gap_open = params->pf_gap_open;
    dp.pf_gap_extend = params->pf_gap_extend;
    dp.temperature = params->temperature;
    dp.w_hmm = params->w_hmm;
    dp.n_gap_classes = params->n_gap_classes;
    dp.alphabet = qp::alphabet_of(params);

    // the pipeline, in stream order on the caller's stream: counters, host
    // data, aligned sequence copy, tables, schedule, the class kernels one
    // after another (each on at most `slots` waves), output scan and gather
    hipLaunchKernelGGL(k_na_clear, dim3(std::min(1024, (kNumInts + 255) / 256)), dim3(256), 0, s, d_ints, kNumInts,
                       out->status);
    NA_TRY(hipGetLastError());
    NA_TRY(put(reinterpret_cast<uint32_t*>(d_params), &dp, sizeof(dp), s));
    NA_TRY(put(reinterpret_cast<uint32_t*>(d_lens), lens, (size_t)n * 4, s));
    hipLaunchKernelGGL(k_na_pad, dim3((unsigned)std::min<int64_t>(1024, (n + 256) / 256)), dim3(256), 0, s, d_lens, n,
                       d_seqa_off);
    NA_TRY(hipGetLastError());
    NA_TRY(qp::scan_i64(d_seqa_off, (int64_t)n + 1, d_scan_tmp, s));
    NA_TRY(qp::launch_stage_seqs(n, qp::alphabet_of(params), d_seqs, d_seq_off, d_lens, d_seqa_off, d_seqa,
                                 d_ints + kIntFlags, s));
    NA_TRY(qp::launch_tables(d_params, d_tab, d_consts, d_col0, mmax, fp64, s));
    NA_TRY(qp::launch_setup(n, d_lens, nullptr, nullptr, nullptr, P, out->pair_i, out->pair_j, out->row_off, d_key,
                            d_ints + kIntHist, out->nnz_off, cmap, s));
    NA_TRY(qp::launch_bins(d_ints + kIntHist, d_bin_start, s));
    NA_TRY(qp::launch_fill_queue(P, d_key, d_bin_start, d_ints + kIntFill, d_queue, s));
    NA_TRY(qp::scan_i64(out->row_off, P + 1, d_scan_tmp, s));
    for (int c = qp::kClasses - 1; c >= 0; --c) {
        if (!cls[c].pairs) continue;
        qp::PairArgs ca = a;
        ca.cls = c;
        ca.cap = cargs[c].cap;
        ca.scratch = d_slots;
        ca.slot_bytes = cargs[c].slot_bytes;
        ca.off_exps = cargs[c].off_exps;
        ca.off_fb = cargs[c].off_fb;
        ca.off_bb = cargs[c].off_bb;
        ca.off_log = cargs[c].off_log;
        ca.spill_band_stride = cargs[c].spill_band_stride;
        ca.exps_band_stride = cargs[c].exps_band_stride;
        ca.bnd_stride = cargs[c].bnd_stride;
        // waves of this class: its occupancy-limited grid, its pair count and
        // the slots that fit in the workspace (the slot area is reused by the
        // next class, which starts after this one on the same stream)
        const int per_cu = ck[c] ? qp::pairs_ck_blocks_per_cu(c) : qp::pairs_blocks_per_cu(c, fp64);
        int64_t grid = std::max<int64_t>(1, (int64_t)std::llround(per_cu * n_cu * frac[c]));
        grid = std::min<int64_t>(grid, (cls[c].pairs + qp::kWavesPerBlock - 1) / qp::kWavesPerBlock);
        grid = std::min<int64_t>(grid, slots / qp::kWavesPerBlock);
        if (ck[c])
            NA_TRY(qp::launch_pairs_ck(c, (int)grid, ca, s));
        else
            NA_TRY(qp::launch_pairs(c, fp64, (int)grid, ca, s));
    }
    NA_TRY(qp::scan_i64(out->nnz_off, P + 1, d_scan_tmp, s));
    NA_TRY(qp::launch_gather(P, out->nnz_off, d_base, d_pool_col, d_pool_val, out->col, out->val, bound, s));
    hipLaunchKernelGGL(k_na_status, dim3(1), dim3(64), 0, s, d_ints + kIntFlags, out->status);
    NA_TRY(hipGetLastError());
    return QP_OK;
}
