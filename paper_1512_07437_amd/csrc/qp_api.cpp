// C ABI of the all-pairs posterior engine: validation, plans (device
// workspace, longest-first schedule, captured HIP graph, timing), the
// blocking host entry points and result transfer.  See include/qp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qp.h"
#include "qp_internal.h"

namespace {

thread_local std::string g_err;

// process-wide tuning table (qp_set_tuning); plans copy it when made
std::mutex g_tuning_mu;
void default_tuning(qp_tuning* t) {
    *t = qp_tuning{};
    for (int r = 0; r < 8; ++r) t->rows_per_lane[r] = r + 1;
    for (int c = 0; c < 9; ++c) {
        t->waves_frac[c] = 1.0;
        t->recompute[c] = c <= qp::kCkMaxClass ? 1 : 0;
    }
    t->concurrent_classes = 1;
    t->orient = 1;
}
qp_tuning g_tuning = [] {
    qp_tuning t;
    default_tuning(&t);
    return t;
}();

qp_status fail(qp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) return fail(QP_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

// Most entries one row of a pair with c columns can keep: the posteriors of
// a row sum to at most one, so at most floor(1/thresh) of them reach the
// threshold; one more covers rounding (the kernels' per-row capacity).
// residue codes of the parameters: 0..alphabet-1 (0 reads as 20)
int alphabet_of(const qp_params* p) { return p->alphabet == 0 ? QP_ALPHA : p->alphabet; }

int64_t row_bound(int32_t c, float thresh) {
    return (int64_t)std::min((double)c, std::floor(1.0 / (double)thresh) + 1.0);
}

constexpr int kNumEventSets = 8;
// layout of the plan's int counters
constexpr int kMaxSide = 3;                           // side streams of concurrent classes
constexpr int kIntHeads = 0;                          // [kClasses] queue heads
constexpr int kIntFlags = 12;                         // overflow flags
constexpr int kIntHist = 16;                          // [kKeyBins]
constexpr int kIntFill = kIntHist + qp::kKeyBins;     // [kKeyBins]
constexpr int kIntPool = kIntFill + qp::kKeyBins;     // 64-bit pool head
constexpr int kNumInts = kIntPool + 2;

// QP_TRACE=1 prints each host step of a call to stderr
bool trace_on() {
    static const bool on = [] {
        const char* v = std::getenv("QP_TRACE");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}
void trace(const char* fmt, ...) {
    if (!trace_on()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[qp] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
    va_end(ap);
}

bool is_sym(const double* a, double tol) {
    for (int i = 0; i < QP_ALPHA; ++i)
        for (int j = i + 1; j < QP_ALPHA; ++j)
            if (std::fabs(a[i * QP_ALPHA + j] - a[j * QP_ALPHA + i]) > tol) return false;
    return true;
}

// check that the current device is a gfx950 GPU
qp_status check_device(int* dev_out, int* n_cu) {
    int dev = 0, count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(QP_EDEVICE, "no HIP device available");
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(QP_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
    *dev_out = dev;
    if (n_cu) *n_cu = prop.multiProcessorCount;
    return QP_OK;
}

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

}  // namespace

qp_status qp::set_error(qp_status st, const char* msg) {
    g_err = msg;
    return st;
}

// ----------------------------------------------------------------- plan
struct qp_plan {
    int device = 0;
    int32_t n = 0;
    int64_t P = 0;
    bool all_pairs = true;
    std::vector<int32_t> lens;
    std::vector<int32_t> list_i, list_j;
    // plain per-pair form: one launch per pair in pair order (no graph);
    // pair_cls holds each pair's kernel class
    bool per_pair = false;
    std::vector<uint8_t> pair_cls;
    // per pair: 1 = swept with the second sequence as rows (empty: none is)
    std::vector<uint8_t> tr;
    uint8_t* d_tr = nullptr;
    // tuning in force when the plan was made
    qp::ClassMap cmap{};
    double waves_frac[qp::kClasses] = {};
    int recompute[qp::kClasses] = {};
    qp_params params{};
    float thresh = 0.f;
    int fp64 = 0;
    int mmax = 1, nmax = 1;
    int64_t total_rows = 0;
    int64_t pool_cap = 0;
    qp::PairArgs args{};  // fields shared by every class launch
    // one persistent launch per kernel class present in the family
    struct ClassPlan {
        int64_t pairs = 0, cells = 0;
        int mmax = 1, nmax = 1, R = 1, nb_max = 1, cap = 1, grid = 0;
        bool ck = false;  // checkpointed form (forward values recomputed)
        qp::PairArgs args{};
        char* d_scratch = nullptr;
    } cls[qp::kClasses];
    int n_side = 0;
    hipStream_t side[kMaxSide] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kMaxSide] = {};
    // marks the end of result copies enqueued on the run stream
    hipEvent_t copy_ev = nullptr;
    // device memory (one allocation each; freed in destroy)
    std::vector<void*> allocs;
    qp::DeviceAllocator dev_alloc{};  // hipMalloc / hipFree when unset
    bool single_stream = false;
    int64_t device_bytes = 0;
    qp::DevParams* d_params = nullptr;
    void* d_tab = nullptr;
    void* d_col0 = nullptr;
    qp::DevConsts* d_consts = nullptr;
    int32_t* d_lens = nullptr;
    // 4-byte aligned, padded copy of the family's residues (the kernels read
    // one sequence per pair through the scalar cache in whole dwords)
    uint8_t* d_seqa = nullptr;
    int64_t* d_seqa_off = nullptr;
    std::vector<int64_t> seqa_off;
    const uint8_t* in_seqs = nullptr;
    const int64_t* in_off = nullptr;
    int32_t* d_list_i = nullptr;
    int32_t* d_list_j = nullptr;
    int32_t* d_pi = nullptr;
    int32_t* d_pj = nullptr;
    int64_t* d_rowoff = nullptr;
    int32_t* d_key = nullptr;
    int* d_ints = nullptr;   // queue heads, flags, hist, bin fill, pool head (as 2 ints)
    int n_ints = 0;
    int* d_bin_start = nullptr;
    int32_t* d_queue = nullptr;
    int32_t* d_rowptr = nullptr;
    int64_t* d_nnz = nullptr;
    int64_t* d_base = nullptr;
    int32_t* d_pool_col = nullptr;
    float* d_pool_val = nullptr;
    int32_t* d_col = nullptr;
    float* d_val = nullptr;
    double* d_dist = nullptr;
    double* d_logz = nullptr;
    int64_t* d_scan_tmp = nullptr;
    // graph and timing
    bool use_graph = true;
    bool graph_broken = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec[kNumEventSets] = {};
    const void* cap_seqs = nullptr;
    const void* cap_off = nullptr;
    hipEvent_t ev[kNumEventSets][4] = {};
    // start / end of each class kernel, recorded on the stream it runs on
    hipEvent_t cev[kNumEventSets][qp::kClasses][2] = {};
    bool ev_pending[kNumEventSets] = {};
    bool ev_cls[kNumEventSets] = {};  // the run on this event set recorded class events
    int run_idx = 0;
    double sum_kernel_ms = 0.0, sum_pipe_ms = 0.0;
    double sum_class_ms[qp::kClasses] = {};
    int64_t n_timed = 0;
    hipStream_t last_stream = nullptr;
    bool ran = false;
    int last_g = -1;     // event set of the last run
    int64_t last_nnz = 0;
};

namespace {

template <typename T>
qp_status dalloc(qp_plan* pl, T** out, int64_t count, int64_t* dry) {
    const int64_t bytes = std::max<int64_t>(count, 1) * (int64_t)sizeof(T);
    if (dry) {  // size accounting only
        *dry += (bytes + 255) & ~int64_t(255);
        *out = nullptr;
        return QP_OK;
    }
    void* p = nullptr;
    if (pl->dev_alloc.alloc) {
        p = pl->dev_alloc.alloc(pl->dev_alloc.ctx, (size_t)bytes);
        if (!p) return fail(QP_ENOMEM, "device allocation of %lld bytes failed", (long long)bytes);
    } else {
        hipError_t e = hipMalloc(&p, (size_t)bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(QP_ENOMEM, "hipMalloc of %lld bytes failed: %s", (long long)bytes, hipGetErrorString(e));
        }
    }
    pl->allocs.push_back(p);
    pl->device_bytes += bytes;
    *out = static_cast<T*>(p);
    return QP_OK;
}

void plan_free_device(qp_plan* pl) {
    for (int g = 0; g < kNumEventSets; ++g) {
        if (pl->exec[g]) hipGraphExecDestroy(pl->exec[g]);
        pl->exec[g] = nullptr;
    }
    for (void* p : pl->allocs) {
        if (pl->dev_alloc.release) pl->dev_alloc.release(pl->dev_alloc.ctx, p);
        else hipFree(p);
    }
    pl->allocs.clear();
    pl->device_bytes = 0;
}

qp_status validate_lens(const int32_t* lens, int32_t n) {
    if (n < 0) return fail(QP_EINVAL, "n = %d < 0", n);
    if (n > 0 && !lens) return fail(QP_EINVAL, "lens is NULL");
    for (int32_t i = 0; i < n; ++i)
        if (lens[i] < 1) return fail(QP_EINVAL, "lens[%d] = %d < 1 (empty sequences are not allowed)", i, lens[i]);
    for (int32_t i = 0; i < n; ++i)
        if (lens[i] > qp::kMaxSeqLen)
            return fail(QP_EINVAL,
                        "lens[%d] = %d > %d: sequences needing more than three row bands are disabled pending "
                        "the cause of a GPU fault on 3000-5000 residue pairs",
                        i, lens[i], qp::kMaxSeqLen);
    return QP_OK;
}

// sizes of one per-wave scratch slot of a kernel class
void size_slot(const qp_plan* pl, qp_plan::ClassPlan* c) {
    qp::slot_layout(c->R, c->mmax, c->nmax, c->nb_max, c->cap, pl->fp64, c->ck, &c->args);
}

}  // namespace

// ------------------------------------------- helpers shared with qp_noalloc
int qp::alphabet_of(const qp_params* p) { return ::alphabet_of(p); }
int64_t qp::row_bound(int32_t cols, float thresh) { return ::row_bound(cols, thresh); }
qp_status qp::validate_lens(const int32_t* lens, int32_t n) { return ::validate_lens(lens, n); }
qp_status qp::check_device(int* dev, int* n_cu) { return ::check_device(dev, n_cu); }
qp_status qp::fail_msg(qp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
void qp::current_tuning(qp::ClassMap* map, double* waves_frac, int* recompute) {
    std::lock_guard<std::mutex> g(g_tuning_mu);
    for (int r = 0; r < qp::kRMax; ++r) map->c[r] = (int8_t)(g_tuning.rows_per_lane[r] - 1);
    for (int c = 0; c < qp::kClasses; ++c) {
        waves_frac[c] = g_tuning.waves_frac[qp::tune_index(c)];
        recompute[c] = g_tuning.recompute[qp::tune_index(c)];
    }
}
void qp::slot_layout(int R, int mmax, int nmax, int nb_max, int cap, int fp64, bool ck, qp::PairArgs* a) {
    const int64_t v2 = fp64 ? 16 : 8;
    const int64_t steps = (int64_t)nmax + qp::kWave - 1;
    if (ck) {
        // per band: the saved forward state of every 8-step block; the
        // forward boundary records of every band; two backward ones
        const int64_t blocks = (steps + qp::kRescaleEvery - 1) / qp::kRescaleEvery;
        a->spill_band_stride = blocks * qp::ck_state_words(R) * qp::kWave;
        a->exps_band_stride = 0;
        a->bnd_stride = nmax + 2;
        int64_t off = align256(nb_max * a->spill_band_stride * 4);
        a->off_exps = off;
        a->off_fb = off;
        off += align256(nb_max * a->bnd_stride * (int64_t)qp::fwd_bnd_bytes(0));
        a->off_bb = off;
        off += align256(2 * a->bnd_stride * (int64_t)qp::bwd_bnd_bytes(0));
        a->off_log = off;
        off += align256((int64_t)mmax * cap * 16);
        a->slot_bytes = off;
        return;
    }
    a->spill_band_stride = steps * qp::kWave * R;
    a->exps_band_stride = ((steps + qp::kRescaleEvery - 1) / qp::kRescaleEvery) * qp::kWave;
    a->bnd_stride = nmax + 2;
    int64_t off = align256(nb_max * a->spill_band_stride * v2);
    a->off_exps = off;
    off += align256(nb_max * a->exps_band_stride * 8);
    a->off_fb = off;
    off += align256(2 * a->bnd_stride * (int64_t)qp::fwd_bnd_bytes(fp64));
    a->off_bb = off;
    off += align256(2 * a->bnd_stride * (int64_t)qp::bwd_bnd_bytes(fp64));
    // hit log: at most cap records of 16 bytes per row
    a->off_log = off;
    off += align256((int64_t)mmax * cap * 16);
    a->slot_bytes = off;
}

// per-class launch arguments: the shared fields plus the class's scratch
static void set_class_args(qp_plan* pl) {
    for (int c = 0; c < qp::kClasses; ++c) {
        qp_plan::ClassPlan& cp = pl->cls[c];
        if (cp.grid == 0) continue;
        qp::PairArgs a = pl->args;
        a.cls = c;
        a.cap = cp.cap;
        a.scratch = cp.d_scratch;
        a.slot_bytes = cp.args.slot_bytes;
        a.off_exps = cp.args.off_exps;
        a.off_fb = cp.args.off_fb;
        a.off_bb = cp.args.off_bb;
        a.off_log = cp.args.off_log;
        a.spill_band_stride = cp.args.spill_band_stride;
        a.exps_band_stride = cp.args.exps_band_stride;
        a.bnd_stride = cp.args.bnd_stride;
        cp.args = a;
    }
}

// allocation of all plan buffers (needs pool_cap and grids); with `dry`
// only adds up the bytes it would allocate
// ns per lane-row-step of each kernel class (C3, each class alone, default
// forms): the cost model that picks a pair's orientation
constexpr double kSlotCost[qp::kClasses] = {4.61, 3.42, 2.89, 2.64, 2.50, 3.27, 3.26, 3.23, 3.42, 3.32, 2.98, 2.82};

// modelled time of sweeping m rows by c columns: per band, c + L - 1 steps
// of 64 lanes x R rows (L lanes in use), times the class's cost per step
static double sweep_cost(int32_t m, int32_t c, const qp::ClassMap& map) {
    const int cls = qp::pair_class(m, map);
    const int R = qp::class_rows_per_lane(cls);
    const int H = qp::kWave * R;
    const int nb = qp::class_banded(cls) ? (m + H - 1) / H : 1;
    double slots = 0.0;
    for (int b = 0; b < nb; ++b) {
        const int rows = std::min(H, m - b * H);
        const int L = (rows + R - 1) / R;
        slots += (double)(c + L - 1) * qp::kWave * R;
    }
    return slots * kSlotCost[cls];
}

// the tables of both models are exactly symmetric (then P(y, x) = P(x, y)^T
// to the last bit of the inputs)
static bool symmetric_tables(const qp_params& p) {
    for (int a = 0; a < QP_ALPHA; ++a)
        for (int b = a + 1; b < QP_ALPHA; ++b)
            if (p.joint[a * QP_ALPHA + b] != p.joint[b * QP_ALPHA + a] ||
                p.score[a * QP_ALPHA + b] != p.score[b * QP_ALPHA + a])
                return false;
    return true;
}

// rows of pair p's sweep (its first sequence's m unless it is transposed)
static int32_t swept_rows(const qp_plan* pl, int64_t p, int32_t m, int32_t c) {
    return !pl->tr.empty() && pl->tr[(size_t)p] ? c : m;
}

// Streams of a plan's classes: with classes side by side, the present
// classes from the largest down are dealt round-robin over min(present,
// kMaxSide) side streams; one after another, they all share the run stream.
// group[c] receives class c's stream, the return value the number of them.
static int stream_groups(const qp_plan* pl, int* group) {
    int np = 0;
    for (int c = qp::kClasses - 1; c >= 0; --c) {
        group[c] = 0;
        if (pl->cls[c].grid > 0) group[c] = np++;
    }
    const int ns = pl->single_stream || np <= 1 ? 1 : std::min(np, kMaxSide);
    for (int c = 0; c < qp::kClasses; ++c) group[c] %= ns;
    return ns;
}

// scratch bytes of the plan's classes (one area per stream)
static int64_t scratch_bytes(const qp_plan* pl, int* n_areas) {
    int group[qp::kClasses];
    int64_t most[kMaxSide] = {};
    const int ng = stream_groups(pl, group);
    for (int c = 0; c < qp::kClasses; ++c)
        if (pl->cls[c].grid > 0)
            most[group[c]] = std::max(most[group[c]], (int64_t)pl->cls[c].grid * qp::kWavesPerBlock *
                                                          pl->cls[c].args.slot_bytes);
    int64_t sum = 0;
    for (int g = 0; g < ng; ++g) sum += most[g];
    if (n_areas) *n_areas = ng;
    return sum;
}

static qp_status plan_alloc_all(qp_plan* pl, int64_t* dry = nullptr) {
    const int64_t P = pl->P;
    qp_status st;
#define ALLOC(ptr, cnt) \
    if ((st = dalloc(pl, &(ptr), (cnt), dry)) != QP_OK) return st
    ALLOC(pl->d_params, 1);
    {
        char* t = nullptr;
        ALLOC(t, (int64_t)qp::kTabRows * qp::kTabW * (pl->fp64 ? 16 : 8));
        pl->d_tab = t;
    }
    {
        char* t = nullptr;
        ALLOC(t, (int64_t)pl->mmax * (int64_t)qp::col0_bytes() + 64);
        pl->d_col0 = t;
    }
    ALLOC(pl->d_consts, 1);
    ALLOC(pl->d_lens, pl->n);
    pl->seqa_off.assign((size_t)pl->n + 1, 0);
    for (int32_t i = 0; i < pl->n; ++i) pl->seqa_off[i + 1] = pl->seqa_off[i] + ((pl->lens[i] + 3) & ~3);
    ALLOC(pl->d_seqa, pl->seqa_off[pl->n] + 4);
    ALLOC(pl->d_seqa_off, pl->n + 1);
    if (!pl->all_pairs) {
        ALLOC(pl->d_list_i, P);
        ALLOC(pl->d_list_j, P);
    }
    if (!pl->tr.empty()) ALLOC(pl->d_tr, P);
    ALLOC(pl->d_pi, P);
    ALLOC(pl->d_pj, P);
    ALLOC(pl->d_rowoff, P + 1);
    ALLOC(pl->d_key, P);
    pl->n_ints = kNumInts;
    ALLOC(pl->d_ints, pl->n_ints);
    ALLOC(pl->d_bin_start, qp::kKeyBins);
    ALLOC(pl->d_queue, P);
    ALLOC(pl->d_rowptr, pl->total_rows);
    ALLOC(pl->d_nnz, P + 1);
    ALLOC(pl->d_base, P);
    ALLOC(pl->d_pool_col, pl->pool_cap);
    ALLOC(pl->d_pool_val, pl->pool_cap);
    ALLOC(pl->d_col, pl->pool_cap);
    ALLOC(pl->d_val, pl->pool_cap);
    ALLOC(pl->d_dist, P);
    ALLOC(pl->d_logz, 2 * P);
    ALLOC(pl->d_scan_tmp, qp::scan_tmp_elems(P + 1) + 8);
    {
        // classes that run one after another on one stream share a scratch
        // area: one area per stream, as large as its largest class's
        int group[qp::kClasses];
        int64_t most[kMaxSide] = {};
        const int ng = stream_groups(pl, group);
        for (int c = 0; c < qp::kClasses; ++c)
            if (pl->cls[c].grid > 0)
                most[group[c]] = std::max(most[group[c]], (int64_t)pl->cls[c].grid * qp::kWavesPerBlock *
                                                              pl->cls[c].args.slot_bytes);
        char* area[kMaxSide] = {};
        for (int g = 0; g < ng; ++g) ALLOC(area[g], most[g]);
        for (int c = 0; c < qp::kClasses; ++c)
            if (pl->cls[c].grid > 0) pl->cls[c].d_scratch = area[group[c]];
    }
#undef ALLOC
    if (dry) return QP_OK;
    HIP_TRY(hipMemcpy(pl->d_lens, pl->lens.data(), sizeof(int32_t) * pl->n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(pl->d_seqa_off, pl->seqa_off.data(), sizeof(int64_t) * (pl->n + 1), hipMemcpyHostToDevice));
    if (!pl->all_pairs) {
        HIP_TRY(hipMemcpy(pl->d_list_i, pl->list_i.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(pl->d_list_j, pl->list_j.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
    }
    if (!pl->tr.empty()) HIP_TRY(hipMemcpy(pl->d_tr, pl->tr.data(), (size_t)P, hipMemcpyHostToDevice));
    qp::DevParams dp{};
    std::memcpy(dp.joint, pl->params.joint, sizeof(dp.joint));
    std::memcpy(dp.score, pl->params.score, sizeof(dp.score));
    for (int k = 0; k < 2; ++k) {
        dp.gap_open[k] = k < pl->params.n_gap_classes ? pl->params.gap_open[k] : 0.0;
        dp.gap_extend[k] = k < pl->params.n_gap_classes ? pl->params.gap_extend[k] : 0.0;
    }
    dp.pf_gap_open = pl->params.pf_gap_open;
    dp.pf_gap_extend = pl->params.pf_gap_extend;
    dp.temperature = pl->params.temperature;
    dp.w_hmm = pl->params.w_hmm;
    dp.n_gap_classes = pl->params.n_gap_classes;
    dp.alphabet = alphabet_of(&pl->params);
    HIP_TRY(hipMemcpy(pl->d_params, &dp, sizeof(dp), hipMemcpyHostToDevice));

    qp::PairArgs& a = pl->args;
    a.lens = pl->d_lens;
    a.seqs = pl->d_seqa;
    a.seq_off = pl->d_seqa_off;
    a.pair_i = pl->d_pi;
    a.pair_j = pl->d_pj;
    a.tr = pl->d_tr;
    a.queue = pl->d_queue;
    a.n_pairs = P;
    a.queue_head = pl->d_ints + kIntHeads;
    a.hist = pl->d_ints + kIntHist;
    a.bin_start = pl->d_bin_start;
    a.tab = pl->d_tab;
    a.col0 = pl->d_col0;
    a.consts = pl->d_consts;
    a.thresh = pl->thresh;
    a.cap_thresh = (int)std::min<double>(qp::kMaxSeqLen + 1, std::floor(1.0 / (double)pl->thresh) + 1.0);
    a.row_off = pl->d_rowoff;
    a.row_ptr = pl->d_rowptr;
    a.pair_nnz = pl->d_nnz;
    a.pair_base = pl->d_base;
    a.pool_col = pl->d_pool_col;
    a.pool_val = pl->d_pool_val;
    a.pool_cap = pl->pool_cap;
    a.pool_head = reinterpret_cast<unsigned long long*>(pl->d_ints + kIntPool);
    a.dist = pl->d_dist;
    a.logz = pl->d_logz;
    a.flags = pl->d_ints + kIntFlags;
    set_class_args(pl);
    return QP_OK;
}

// record a timing event; inside a graph capture it must be an external
// event node, otherwise it only orders the capture
static hipError_t record(hipEvent_t e, hipStream_t s, bool capturing) {
    return capturing ? hipEventRecordWithFlags(e, s, hipEventRecordExternal) : hipEventRecord(e, s);
}

// enqueue every step of the pipeline on s; events optional
static qp_status enqueue_pipeline(qp_plan* pl, hipStream_t s, int ev_set, bool capturing = false) {
    const int64_t P = pl->P;
    hipEvent_t* ev = ev_set >= 0 ? pl->ev[ev_set] : nullptr;
    if (ev) HIP_TRY(record(ev[0], s, capturing));
    HIP_TRY(qp::launch_reset(pl->d_ints, pl->n_ints, s));
    HIP_TRY(qp::launch_stage_seqs(pl->n, alphabet_of(&pl->params), pl->in_seqs, pl->in_off, pl->d_lens, pl->d_seqa_off, pl->d_seqa,
                                  pl->d_ints + kIntFlags, s));
    HIP_TRY(qp::launch_tables(pl->d_params, pl->d_tab, pl->d_consts, pl->d_col0, pl->mmax, pl->fp64, s));
    HIP_TRY(qp::launch_setup(pl->n, pl->d_lens, pl->d_list_i, pl->d_list_j, pl->d_tr, P, pl->d_pi, pl->d_pj, pl->d_rowoff,
                             pl->d_key, pl->d_ints + kIntHist, pl->d_nnz, pl->cmap, s));
    HIP_TRY(qp::launch_bins(pl->d_ints + kIntHist, pl->d_bin_start, s));
    HIP_TRY(qp::launch_fill_queue(P, pl->d_key, pl->d_bin_start, pl->d_ints + kIntFill, pl->d_queue, s));
    HIP_TRY(qp::scan_i64(pl->d_rowoff, P + 1, pl->d_scan_tmp, s));
    if (ev) HIP_TRY(record(ev[1], s, capturing));
    if (pl->per_pair) {
        for (int64_t p = 0; p < P; ++p) {
            const int c = pl->pair_cls[p];
            if (pl->cls[c].ck)
                HIP_TRY(qp::launch_pair_one_ck(c, p, pl->cls[c].args, s));
            else
                HIP_TRY(qp::launch_pair_one(c, pl->fp64, p, pl->cls[c].args, s));
        }
        if (ev) HIP_TRY(record(ev[2], s, capturing));
        HIP_TRY(qp::scan_i64(pl->d_nnz, P + 1, pl->d_scan_tmp, s));
        HIP_TRY(qp::launch_gather(P, pl->d_nnz, pl->d_base, pl->d_pool_col, pl->d_pool_val, pl->d_col,
                                  pl->d_val, pl->pool_cap, s));
        if (ev) HIP_TRY(record(ev[3], s, capturing));
        return QP_OK;
    }
    // the kernel classes run concurrently on the side streams (fork / join)
    int present[qp::kClasses], np = 0;
    for (int c = qp::kClasses - 1; c >= 0; --c)
        if (pl->cls[c].grid > 0) present[np++] = c;
    auto launch_class = [&](int c, hipStream_t cs) -> qp_status {
        if (ev) HIP_TRY(record(pl->cev[ev_set][c][0], cs, capturing));
        if (pl->cls[c].ck)
            HIP_TRY(qp::launch_pairs_ck(c, pl->cls[c].grid, pl->cls[c].args, cs));
        else
            HIP_TRY(qp::launch_pairs(c, pl->fp64, pl->cls[c].grid, pl->cls[c].args, cs));
        if (ev) HIP_TRY(record(pl->cev[ev_set][c][1], cs, capturing));
        return QP_OK;
    };
    qp_status cst;
    if (np == 1 || pl->n_side == 0) {
        for (int q = 0; q < np; ++q)
            if ((cst = launch_class(present[q], s)) != QP_OK) return cst;
    } else {
        HIP_TRY(hipEventRecord(pl->fork_ev, s));
        const int ns = std::min(np, pl->n_side);
        for (int q = 0; q < ns; ++q) HIP_TRY(hipStreamWaitEvent(pl->side[q], pl->fork_ev, 0));
        for (int q = 0; q < np; ++q)
            if ((cst = launch_class(present[q], pl->side[q % ns])) != QP_OK) return cst;
        for (int q = 0; q < ns; ++q) {
            HIP_TRY(hipEventRecord(pl->join_ev[q], pl->side[q]));
            HIP_TRY(hipStreamWaitEvent(s, pl->join_ev[q], 0));
        }
    }
    if (ev) HIP_TRY(record(ev[2], s, capturing));
    HIP_TRY(qp::scan_i64(pl->d_nnz, P + 1, pl->d_scan_tmp, s));
    HIP_TRY(qp::launch_gather(P, pl->d_nnz, pl->d_base, pl->d_pool_col, pl->d_pool_val, pl->d_col,
                              pl->d_val, pl->pool_cap, s));
    if (ev) HIP_TRY(record(ev[3], s, capturing));
    return QP_OK;
}

static qp_status capture_graphs(qp_plan* pl) {
    // a launch of these graphs may still be in flight: it ends before any of
    // them goes (runs of a plan are ordered one after the other, so the last
    // run's end covers every earlier one)
    if (pl->ran && pl->last_g >= 0) {
        hipError_t e = hipEventSynchronize(pl->ev[pl->last_g][3]);
        if (e != hipSuccess) return fail(QP_EDEVICE, "waiting for the previous run: %s", hipGetErrorString(e));
    }
    for (int g = 0; g < kNumEventSets; ++g) {
        if (pl->exec[g]) {
            hipGraphExecDestroy(pl->exec[g]);
            pl->exec[g] = nullptr;
        }
    }
    for (int g = 0; g < kNumEventSets; ++g) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(QP_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        qp_status st = enqueue_pipeline(pl, pl->cap_stream, g, true);
        e = hipStreamEndCapture(pl->cap_stream, &graph);
        if (st != QP_OK) {
            if (graph) hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(QP_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&pl->exec[g], graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(QP_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return QP_OK;
}

static void collect_timing(qp_plan* pl) {
    for (int g = 0; g < kNumEventSets; ++g) {
        if (!pl->ev_pending[g]) continue;
        float k = 0.f, p = 0.f;
        if (hipEventElapsedTime(&k, pl->ev[g][1], pl->ev[g][2]) == hipSuccess &&
            hipEventElapsedTime(&p, pl->ev[g][0], pl->ev[g][3]) == hipSuccess) {
            pl->sum_kernel_ms += k;
            pl->sum_pipe_ms += p;
            pl->n_timed += 1;
            for (int c = 0; c < qp::kClasses && pl->ev_cls[g]; ++c) {
                float ck = 0.f;
                if (pl->cls[c].grid > 0 &&
                    hipEventElapsedTime(&ck, pl->cev[g][c][0], pl->cev[g][c][1]) == hipSuccess)
                    pl->sum_class_ms[c] += ck;
                else
                    (void)hipGetLastError();
            }
        } else {
            (void)hipGetLastError();
        }
        pl->ev_pending[g] = false;
    }
}

extern "C" {

int32_t qp_version(void) { return (1 << 16) | 0; }

const char* qp_last_error(void) { return g_err.c_str(); }

void qp_params_default(qp_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_gap_classes = 2;
    p->gap_open[0] = 0.02;
    p->gap_open[1] = 0.005;
    p->gap_extend[0] = 0.5;
    p->gap_extend[1] = 0.9;
    p->pf_gap_open = -12.0;
    p->pf_gap_extend = -1.0;
    p->temperature = 5.0;
    p->w_hmm = 0.5;
    p->precision = QP_FP32_SCALED;
    p->alphabet = QP_ALPHA;
}

qp_status qp_params_check(const qp_params* p) {
    if (!p) return fail(QP_EINVAL, "params is NULL");
    const int A = alphabet_of(p);
    if (A < 2 || A > QP_ALPHA) return fail(QP_EINVAL, "alphabet = %d is not in [2, %d]", p->alphabet, QP_ALPHA);
    double s = 0.0;
    for (int i = 0; i < QP_ALPHA * QP_ALPHA; ++i) {
        const double v = p->joint[i];
        if (i / QP_ALPHA < A && i % QP_ALPHA < A) {
            if (!(v > 0.0 && v < 1.0)) return fail(QP_EINVAL, "joint[%d] = %g is not in (0,1)", i, v);
        } else if (v != 0.0) {
            return fail(QP_EINVAL, "joint[%d] = %g lies outside the %d-letter alphabet and must be 0", i, v, A);
        }
        s += v;
        if (!std::isfinite(p->score[i])) return fail(QP_EINVAL, "score[%d] is not finite", i);
    }
    if (std::fabs(s - 1.0) > 1e-9) return fail(QP_EINVAL, "joint sums to %.17g, not 1", s);
    if (!is_sym(p->joint, 1e-12)) return fail(QP_EINVAL, "joint is not symmetric");
    if (!is_sym(p->score, 1e-12)) return fail(QP_EINVAL, "score is not symmetric");
    if (p->n_gap_classes < 1 || p->n_gap_classes > QP_MAX_GAP_CLASSES)
        return fail(QP_EINVAL, "n_gap_classes = %d (must be 1 or 2)", p->n_gap_classes);
    double tau = 1.0;
    for (int k = 0; k < p->n_gap_classes; ++k) {
        if (!(p->gap_open[k] > 0.0 && p->gap_open[k] < 0.5))
            return fail(QP_EINVAL, "gap_open[%d] = %g is not in (0, 0.5)", k, p->gap_open[k]);
        if (!(p->gap_extend[k] >= 0.0 && p->gap_extend[k] < 1.0))
            return fail(QP_EINVAL, "gap_extend[%d] = %g is not in [0, 1)", k, p->gap_extend[k]);
        tau -= 2.0 * p->gap_open[k];
    }
    if (!(tau > 0.0)) return fail(QP_EINVAL, "1 - 2*sum(gap_open) = %g must be > 0", tau);
    if (!(p->temperature > 0.0) || !std::isfinite(p->temperature))
        return fail(QP_EINVAL, "temperature = %g must be > 0", p->temperature);
    if (!std::isfinite(p->pf_gap_open) || !std::isfinite(p->pf_gap_extend))
        return fail(QP_EINVAL, "PF gap scores must be finite");
    if (!(p->w_hmm >= 0.0 && p->w_hmm <= 1.0)) return fail(QP_EINVAL, "w_hmm = %g is not in [0,1]", p->w_hmm);
    if (p->precision != QP_FP32_SCALED && p->precision != QP_FP64)
        return fail(QP_EINVAL, "precision = %d is unknown", p->precision);
    // the kernels hold per-residue weights in the working precision
    const double lim = p->precision == QP_FP64 ? 600.0 : 80.0;
    for (int i = 0; i < QP_ALPHA * QP_ALPHA; ++i)
        if (std::fabs(p->score[i] / p->temperature) > lim)
            return fail(QP_EINVAL, "score[%d]/T = %g is outside the representable weight range", i,
                        p->score[i] / p->temperature);
    if (std::fabs(p->pf_gap_open / p->temperature) > lim || std::fabs(p->pf_gap_extend / p->temperature) > lim)
        return fail(QP_EINVAL, "PF gap score / T is outside the representable weight range");
    return QP_OK;
}

}  // extern "C"

// Shape of a plan: validation, per-class work, grids and sizes; no device
// memory yet.  wave_budget > 0 caps the resident waves of all its classes.
qp_status qp::plan_shape(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                         int64_t n_pairs, const qp_params* params, float thresh, int64_t nnz_capacity,
                         int64_t wave_budget, qp_plan** plan) {
    if (!plan) return fail(QP_EINVAL, "plan is NULL");
    *plan = nullptr;
    qp_status st = validate_lens(lens, n);
    if (st != QP_OK) return st;
    if ((st = qp_params_check(params)) != QP_OK) return st;
    if (!(thresh > 0.0f && thresh <= 1.0f)) return fail(QP_EINVAL, "thresh = %g is not in (0, 1]", (double)thresh);
    if (nnz_capacity < -1) return fail(QP_EINVAL, "nnz_capacity = %lld < -1", (long long)nnz_capacity);
    const bool all = pair_i == nullptr && pair_j == nullptr;
    if (!all) {
        if (!pair_i || !pair_j) return fail(QP_EINVAL, "pair_i and pair_j must both be given");
        if (n_pairs < 0) return fail(QP_EINVAL, "n_pairs < 0");
        for (int64_t k = 0; k < n_pairs; ++k) {
            if (pair_i[k] < 0 || pair_i[k] >= n || pair_j[k] < 0 || pair_j[k] >= n)
                return fail(QP_EINVAL, "pair %lld = (%d, %d) is out of range", (long long)k, pair_i[k], pair_j[k]);
            if (pair_i[k] == pair_j[k])
                return fail(QP_EINVAL, "pair %lld pairs sequence %d with itself", (long long)k, pair_i[k]);
        }
    }
    const int64_t P = all ? (int64_t)n * (n - 1) / 2 : n_pairs;
    if (P > INT32_MAX) return fail(QP_EINVAL, "%lld pairs exceed the 2^31 limit of one plan", (long long)P);
    int dev = 0, n_cu = 0;
    if ((st = check_device(&dev, &n_cu)) != QP_OK) return st;

    qp_plan* pl = new (std::nothrow) qp_plan();
    if (!pl) return fail(QP_ENOMEM, "out of host memory");
    pl->device = dev;
    pl->n = n;
    pl->P = P;
    pl->all_pairs = all;
    pl->lens.assign(lens, lens + n);
    bool orient = false;
    {
        std::lock_guard<std::mutex> g(g_tuning_mu);
        for (int r = 0; r < qp::kRMax; ++r) pl->cmap.c[r] = (int8_t)(g_tuning.rows_per_lane[r] - 1);
        for (int c = 0; c < qp::kClasses; ++c) {
            pl->waves_frac[c] = g_tuning.waves_frac[qp::tune_index(c)];
            pl->recompute[c] = g_tuning.recompute[qp::tune_index(c)];
        }
        pl->single_stream = g_tuning.concurrent_classes == 0;
        orient = g_tuning.orient != 0;
    }
    if (!all) {
        pl->list_i.assign(pair_i, pair_i + P);
        pl->list_j.assign(pair_j, pair_j + P);
    }
    pl->params = *params;
    pl->thresh = thresh;
    pl->fp64 = params->precision == QP_FP64 ? 1 : 0;

    // shape of the work per kernel class: pairs, cells, longest rows / columns
    // sparse-output estimate: 16 entries per row (8 when that pool would
    // not fit in an eighth of the free device memory), at most 1/thresh
    int64_t rows = 0, est = 0, est_lo = 0, bound = 0;
    const double inv = std::floor(1.0 / (double)thresh);
    const int per_row = (int)std::max(1.0, std::min(16.0, inv));
    const int per_row_lo = (int)std::max(1.0, std::min(8.0, inv));
    // orientation: with symmetric model tables the posterior matrix of (y, x)
    // is the transpose of (x, y)'s, so a pair may be swept with either
    // sequence as rows; each pair takes the orientation of the lower
    // modelled cost, its output rows staying the first sequence's
    const bool may_transpose = orient && symmetric_tables(*params);
    std::vector<uint8_t> tr((size_t)(may_transpose ? P : 0), 0);
    bool any_tr = false;
    int64_t q = 0;
    auto count = [&](int32_t m, int32_t c) {
        const bool t = may_transpose && sweep_cost(c, m, pl->cmap) < sweep_cost(m, c, pl->cmap);
        if (t) {
            tr[(size_t)q] = 1;
            any_tr = true;
        }
        ++q;
        const int32_t ms = t ? c : m, cs = t ? m : c;  // rows and columns of the sweep
        qp_plan::ClassPlan& cp = pl->cls[qp::pair_class(ms, pl->cmap)];
        cp.pairs += 1;
        cp.cells += (int64_t)m * c;
        cp.mmax = std::max(cp.mmax, ms);
        cp.nmax = std::max(cp.nmax, cs);
        pl->mmax = std::max(pl->mmax, ms);
        pl->nmax = std::max(pl->nmax, cs);
        rows += m + 1;
        est += (int64_t)m * std::min(per_row, c);
        est_lo += (int64_t)m * std::min(per_row_lo, c);
        bound += (int64_t)m * row_bound(c, thresh);
    };
    if (all) {
        for (int32_t i = 0; i + 1 < n; ++i)
            for (int32_t j = i + 1; j < n; ++j) count(lens[i], lens[j]);
    } else {
        for (int64_t k = 0; k < P; ++k) count(lens[pair_i[k]], lens[pair_j[k]]);
    }
    if (any_tr) pl->tr.swap(tr);
    pl->total_rows = rows;

    // persistent grid per class: enough waves to fill every SIMD at the
    // kernel's occupancy, bounded by the class's pair count; all classes
    // together stay within half of the free device memory
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = (size_t)64 << 30;
    }
    // the pool and the gathered output hold four 4-byte arrays of this size
    if (16 * est > (int64_t)(free_b / 8)) est = est_lo;
    pl->pool_cap = nnz_capacity > 0    ? nnz_capacity
                   : nnz_capacity == -1 ? std::max<int64_t>(bound, 1)
                                        : std::max<int64_t>(est + 1024, 1024);
    for (int c = 0; c < qp::kClasses; ++c) {
        qp_plan::ClassPlan& cp = pl->cls[c];
        if (cp.pairs == 0) continue;
        cp.ck = !pl->fp64 && pl->recompute[c] != 0;
        cp.R = qp::class_rows(c, cp.ck);
        const int H = qp::kWave * cp.R;
        cp.nb_max = qp::class_banded(c) ? (cp.mmax + H - 1) / H : 1;
        cp.cap = (int)std::max(1.0, std::min((double)cp.nmax, inv + 1.0));
        size_slot(pl, &cp);
        const int per_cu = cp.ck ? qp::pairs_ck_blocks_per_cu(c) : qp::pairs_blocks_per_cu(c, pl->fp64);
        int64_t grid = std::max<int64_t>(1, (int64_t)std::llround(per_cu * n_cu * pl->waves_frac[c]));
        grid = std::min<int64_t>(grid, std::max<int64_t>(1, (cp.pairs + qp::kWavesPerBlock - 1) / qp::kWavesPerBlock));
        cp.grid = (int)grid;
    }
    const int64_t want_bytes = scratch_bytes(pl, nullptr);
    const int64_t budget = (int64_t)(free_b / 2);
    if (want_bytes > budget) {
        const double f = (double)budget / (double)want_bytes;
        for (int c = 0; c < qp::kClasses; ++c)
            if (pl->cls[c].grid > 0) pl->cls[c].grid = std::max(1, (int)(pl->cls[c].grid * f));
    }
    // a wave budget bounds each class kernel on its own (the serving loop runs
    // a family's classes one after the other on the family's stream)
    if (wave_budget > 0) {
        const int64_t max_blocks = std::max<int64_t>(1, wave_budget / qp::kWavesPerBlock);
        for (int c = 0; c < qp::kClasses; ++c)
            if (pl->cls[c].grid > max_blocks) pl->cls[c].grid = (int)max_blocks;
    }
    *plan = pl;
    return QP_OK;
}

// sparse entries produced by the plan's last synchronised run
int64_t qp::plan_last_nnz(const qp_plan* pl) { return pl ? pl->last_nnz : 0; }

void qp::plan_set_allocator(qp_plan* pl, const qp::DeviceAllocator& a) {
    if (pl) pl->dev_alloc = a;
}

void qp::plan_set_single_stream(qp_plan* pl, bool on) {
    if (pl) pl->single_stream = on;
}

// copy the last run's outputs to a library-owned host result
qp_status qp::plan_download(qp_plan* pl, qp_result** out, qp::Staging* stg) {
    if (!out) return fail(QP_EINVAL, "out is NULL");
    *out = nullptr;
    qp_device_result d;
    qp_status st = qp_plan_sync(pl, &d);
    if (st != QP_OK) return st;
    const int64_t P = pl->P;
    qp_result* r = qp::result_alloc(pl->n, P, pl->total_rows, d.nnz);
    if (!r) return fail(QP_ENOMEM, "out of host memory");
    r->thresh = pl->thresh;
    if (P == 0) {
        *out = r;
        return QP_OK;
    }
    // pinned results take the copies directly; pageable ones go through the
    // staging buffer, if there is one
    if (qp::result_pinned(r)) stg = nullptr;
    hipError_t e = hipSuccess;
    // staged copies: chunk k goes through half k % 2; a half is emptied
    // (its copy waited for, then copied out on the host) before it is reused
    struct Pending {
        char* dst = nullptr;
        size_t len = 0;
    } pend[2];
    int half_k = 0;
    auto drain = [&](int k) {
        if (e != hipSuccess || !pend[k].dst) return;
        e = hipEventSynchronize(stg->ev[k]);
        if (e == hipSuccess) std::memcpy(pend[k].dst, stg->buf + (size_t)k * stg->half, pend[k].len);
        pend[k].dst = nullptr;
    };
    auto cp = [&](void* dst, const void* src, size_t b) {
        if (e != hipSuccess || !b) return;
        if (!stg) {
            e = hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, pl->last_stream);
            return;
        }
        for (size_t off = 0; off < b && e == hipSuccess; off += stg->half) {
            const size_t len = std::min(stg->half, b - off);
            drain(half_k);
            if (e != hipSuccess) return;
            e = hipMemcpyAsync(stg->buf + (size_t)half_k * stg->half, static_cast<const char*>(src) + off, len,
                               hipMemcpyDeviceToHost, pl->last_stream);
            if (e == hipSuccess) e = hipEventRecord(stg->ev[half_k], pl->last_stream);
            pend[half_k].dst = static_cast<char*>(dst) + off;
            pend[half_k].len = len;
            half_k ^= 1;
        }
    };
    cp(r->pair_i, d.pair_i, sizeof(int32_t) * P);
    cp(r->pair_j, d.pair_j, sizeof(int32_t) * P);
    cp(r->row_off, d.row_off, sizeof(int64_t) * (P + 1));
    cp(r->row_ptr, d.row_ptr, sizeof(int32_t) * pl->total_rows);
    cp(r->nnz_off, d.nnz_off, sizeof(int64_t) * (P + 1));
    cp(r->col, d.col, sizeof(int32_t) * d.nnz);
    cp(r->val, d.val, sizeof(float) * d.nnz);
    cp(r->dist, d.dist, sizeof(double) * P);
    cp(r->log_z, d.log_z, sizeof(double) * 2 * P);
    if (stg) {
        drain(half_k);  // the older pending half first
        drain(half_k ^ 1);
    } else {
        if (e == hipSuccess) e = hipEventRecord(pl->copy_ev, pl->last_stream);
        if (e == hipSuccess) e = hipEventSynchronize(pl->copy_ev);
    }
    if (e != hipSuccess) {
        qp_result_free(r);
        return fail(QP_EDEVICE, "device-to-host copy failed: %s", hipGetErrorString(e));
    }
    collect_timing(pl);
    r->device_ms = pl->n_timed ? pl->sum_pipe_ms / pl->n_timed : 0.0;
    r->thresh = pl->thresh;
    *out = r;
    return QP_OK;
}

// device bytes a shaped plan will hold
int64_t qp::plan_bytes(qp_plan* pl) {
    int64_t b = 0;
    plan_alloc_all(pl, &b);
    return b;
}

// allocate a shaped plan's device memory, streams and events
qp_status qp::plan_materialize(qp_plan* pl) {
    qp_status st;
    if ((st = plan_alloc_all(pl)) != QP_OK) {
        plan_free_device(pl);
        return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->copy_ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        for (int g = 0; g < kNumEventSets && e == hipSuccess; ++g) {
            for (int q = 0; q < 4 && e == hipSuccess; ++q) e = hipEventCreate(&pl->ev[g][q]);
            for (int c = 0; c < qp::kClasses && e == hipSuccess; ++c)
                if (pl->cls[c].grid > 0)
                    for (int q = 0; q < 2 && e == hipSuccess; ++q) e = hipEventCreate(&pl->cev[g][c][q]);
        }
    }
    int n_present = 0;
    for (int c = 0; c < qp::kClasses; ++c) n_present += pl->cls[c].grid > 0;
    if (e == hipSuccess && n_present > 1 && !pl->single_stream) {
        pl->n_side = std::min(n_present, kMaxSide);
        e = hipEventCreateWithFlags(&pl->fork_ev, hipEventDisableTiming);
        for (int q = 0; q < pl->n_side && e == hipSuccess; ++q) {
            e = hipStreamCreateWithFlags(&pl->side[q], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join_ev[q], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) return fail(QP_EDEVICE, "stream/event creation failed: %s", hipGetErrorString(e));
    if (trace_on()) {
        trace("plan: n=%d pairs=%lld mmax=%d nmax=%d pool=%lld fp64=%d", pl->n, (long long)pl->P, pl->mmax, pl->nmax,
              (long long)pl->pool_cap, pl->fp64);
        for (int c = 0; c < qp::kClasses; ++c)
            if (pl->cls[c].grid > 0)
                trace("  class %d: R=%d bands<=%d pairs=%lld cells=%lld grid=%d slot=%lld B cap=%d", c,
                      pl->cls[c].R, pl->cls[c].nb_max, (long long)pl->cls[c].pairs, (long long)pl->cls[c].cells,
                      pl->cls[c].grid, (long long)pl->cls[c].args.slot_bytes, pl->cls[c].cap);
    }
    return QP_OK;
}

extern "C" {

qp_status qp_plan_create(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                         int64_t n_pairs, const qp_params* params, float thresh, int64_t nnz_capacity,
                         qp_plan** plan) {
    qp_plan* pl = nullptr;
    qp_status st = qp::plan_shape(lens, n, pair_i, pair_j, n_pairs, params, thresh, nnz_capacity, 0, &pl);
    if (st != QP_OK) return st;
    if ((st = qp::plan_materialize(pl)) != QP_OK) {
        std::string keep = g_err;
        qp_plan_destroy(pl);
        g_err = keep;
        return st;
    }
    *plan = pl;
    return QP_OK;
}

qp_status qp_plan_run(qp_plan* pl, const uint8_t* d_seqs, const int64_t* d_seq_off, void* stream) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    if (pl->n > 0 && (!d_seqs || !d_seq_off)) return fail(QP_EINVAL, "device sequence pointers are NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(pl->device));
    // results of the previous run must be read before its events are reused
    const int g = pl->run_idx % kNumEventSets;
    if (pl->ev_pending[g]) {
        HIP_TRY(hipEventSynchronize(pl->ev[g][3]));
        collect_timing(pl);
    }
    // a run on another stream than the previous one starts after it: both
    // use the same workspace and outputs
    if (pl->ran && pl->last_g >= 0 && s != pl->last_stream) HIP_TRY(hipStreamWaitEvent(s, pl->ev[pl->last_g][3], 0));
    pl->in_seqs = d_seqs;
    pl->in_off = d_seq_off;
    pl->last_stream = s;
    pl->ev_cls[g] = !pl->per_pair;  // per-pair runs record no class events
    pl->ran = true;
    if (pl->P == 0) return QP_OK;
    if (pl->use_graph && !pl->graph_broken && !pl->per_pair) {
        if (pl->cap_seqs != d_seqs || pl->cap_off != d_seq_off || !pl->exec[0]) {
            trace("run: capturing graphs");
            qp_status st = capture_graphs(pl);
            trace("run: capture %s%s", st == QP_OK ? "ok" : "failed: ", st == QP_OK ? "" : g_err.c_str());
            if (st != QP_OK) {
                pl->graph_broken = true;  // fall back to eager launches
                (void)hipGetLastError();
            } else {
                pl->cap_seqs = d_seqs;
                pl->cap_off = d_seq_off;
            }
        }
        if (!pl->graph_broken) {
            trace("run: graph %d", g);
            HIP_TRY(hipGraphLaunch(pl->exec[g], s));
            pl->ev_pending[g] = true;
            pl->last_g = g;
            pl->run_idx++;
            return QP_OK;
        }
    }
    trace("run: eager (event set %d)", g);
    qp_status st = enqueue_pipeline(pl, s, g);
    if (st != QP_OK) return st;
    pl->ev_pending[g] = true;
    pl->last_g = g;
    pl->run_idx++;
    return QP_OK;
}

// (rows, columns) of every pair of a family or pair list, after validation
static qp_status visit_pairs(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                             int64_t n_pairs, const std::function<void(int32_t, int32_t)>& f) {
    qp_status st = validate_lens(lens, n);
    if (st != QP_OK) return st;
    if (pair_i == nullptr && pair_j == nullptr) {
        for (int32_t i = 0; i + 1 < n; ++i)
            for (int32_t j = i + 1; j < n; ++j) f(lens[i], lens[j]);
        return QP_OK;
    }
    if (!pair_i || !pair_j) return fail(QP_EINVAL, "pair_i and pair_j must both be given");
    if (n_pairs < 0) return fail(QP_EINVAL, "n_pairs < 0");
    for (int64_t k = 0; k < n_pairs; ++k)
        if (pair_i[k] < 0 || pair_i[k] >= n || pair_j[k] < 0 || pair_j[k] >= n || pair_i[k] == pair_j[k])
            return fail(QP_EINVAL, "pair %lld = (%d, %d) is not a pair of two sequences of the family", (long long)k,
                        pair_i[k], pair_j[k]);
    for (int64_t k = 0; k < n_pairs; ++k) f(lens[pair_i[k]], lens[pair_j[k]]);
    return QP_OK;
}

qp_status qp_output_bound(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                          int64_t n_pairs, float thresh, int64_t* entries) {
    if (!entries) return fail(QP_EINVAL, "entries is NULL");
    if (!(thresh > 0.0f && thresh <= 1.0f)) return fail(QP_EINVAL, "thresh = %g is not in (0, 1]", (double)thresh);
    int64_t total = 0;
    qp_status st = visit_pairs(lens, n, pair_i, pair_j, n_pairs,
                               [&](int32_t m, int32_t c) { total += (int64_t)m * row_bound(c, thresh); });
    if (st != QP_OK) return st;
    *entries = total;
    return QP_OK;
}

qp_status qp_threshold_for_budget(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                                  int64_t n_pairs, int64_t max_entries, float* thresh) {
    if (!thresh) return fail(QP_EINVAL, "thresh is NULL");
    std::vector<std::pair<int32_t, int32_t>> shapes;
    int32_t cmax = 1;
    qp_status st = visit_pairs(lens, n, pair_i, pair_j, n_pairs, [&](int32_t m, int32_t c) {
        shapes.emplace_back(m, c);
        cmax = std::max(cmax, c);
    });
    if (st != QP_OK) return st;
    // entries when every row keeps at most K: non-decreasing in K
    auto at = [&](int64_t K) {
        int64_t t = 0;
        for (const auto& sc : shapes) t += (int64_t)sc.first * std::min<int64_t>(sc.second, K);
        return t;
    };
    // thresh = 1 still leaves two per row (one entry, plus the rounding slack)
    if (at(2) > max_entries)
        return fail(QP_ENOSPC, "even thresh = 1 may need %lld entries, more than %lld", (long long)at(2),
                    (long long)max_entries);
    // the largest row capacity K that fits (beyond the widest pair nothing changes)
    int64_t lo = 2, hi = std::max<int64_t>(2, cmax);
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (at(mid) <= max_entries)
            lo = mid;
        else
            hi = mid - 1;
    }
    // the smallest threshold whose row capacity floor(1/t) + 1 is at most lo
    float t = std::min(1.0f, (float)(1.0 / (double)lo));
    while (t < 1.0f && std::floor(1.0 / (double)t) + 1.0 > (double)lo) t = std::nextafter(t, 2.0f);
    float below = std::nextafter(t, 0.0f);
    while (below > 0.0f && std::floor(1.0 / (double)below) + 1.0 <= (double)lo) {
        t = below;
        below = std::nextafter(t, 0.0f);
    }
    *thresh = t;
    return QP_OK;
}

qp_status qp_set_tuning(const qp_tuning* t) {
    qp_tuning v{};
    if (!t) {
        default_tuning(&v);
    } else {
        for (int c = 0; c < 9; ++c) {
            if (t->recompute[c] != 0 && t->recompute[c] != 1)
                return fail(QP_EINVAL, "recompute[%d] = %d is not 0 or 1", c, t->recompute[c]);
            if (t->recompute[c] && c > qp::kCkMaxClass && c != qp::kBandClass)
                return fail(QP_EINVAL, "recompute[%d] = 1: the checkpointed form exists for classes 0..%d and %d only",
                            c, qp::kCkMaxClass, qp::kBandClass);
        }
        for (int r = 0; r < 8; ++r)
            if (t->rows_per_lane[r] < r + 1 || t->rows_per_lane[r] > 8)
                return fail(QP_EINVAL, "rows_per_lane[%d] = %d is not in [%d, 8]", r, t->rows_per_lane[r], r + 1);
        for (int c = 0; c < 9; ++c)
            if (!(t->waves_frac[c] > 0.0 && t->waves_frac[c] <= 1.0))
                return fail(QP_EINVAL, "waves_frac[%d] = %g is not in (0, 1]", c, t->waves_frac[c]);
        if (t->concurrent_classes != 0 && t->concurrent_classes != 1)
            return fail(QP_EINVAL, "concurrent_classes = %d is not 0 or 1", t->concurrent_classes);
        if (t->orient != 0 && t->orient != 1) return fail(QP_EINVAL, "orient = %d is not 0 or 1", t->orient);
        v = *t;
    }
    std::lock_guard<std::mutex> g(g_tuning_mu);
    g_tuning = v;
    return QP_OK;
}

qp_status qp_get_tuning(qp_tuning* t) {
    if (!t) return fail(QP_EINVAL, "t is NULL");
    std::lock_guard<std::mutex> g(g_tuning_mu);
    *t = g_tuning;
    return QP_OK;
}

qp_status qp_plan_set_per_pair(qp_plan* pl, int32_t on) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    if (on && pl->pair_cls.size() != (size_t)pl->P) {
        try {
            pl->pair_cls.resize((size_t)pl->P);
        } catch (const std::bad_alloc&) {
            return fail(QP_ENOMEM, "out of host memory");
        }
        int64_t p = 0;
        if (pl->all_pairs) {
            for (int32_t i = 0; i + 1 < pl->n; ++i)
                for (int32_t j = i + 1; j < pl->n; ++j, ++p)
                    pl->pair_cls[p] = (uint8_t)qp::pair_class(swept_rows(pl, p, pl->lens[i], pl->lens[j]), pl->cmap);
        } else {
            for (; p < pl->P; ++p)
                pl->pair_cls[p] = (uint8_t)qp::pair_class(
                    swept_rows(pl, p, pl->lens[pl->list_i[p]], pl->lens[pl->list_j[p]]), pl->cmap);
        }
    }
    pl->per_pair = on != 0;
    return QP_OK;
}

qp_status qp_plan_sync(qp_plan* pl, qp_device_result* res) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    if (!pl->ran) return fail(QP_EINVAL, "plan has not been run");
    HIP_TRY(hipSetDevice(pl->device));
    trace("sync: waiting");
    // the plan's own end event: other work queued behind it on the same
    // stream (other families) is not waited for
    if (pl->last_g >= 0 && pl->P > 0)
        HIP_TRY(hipEventSynchronize(pl->ev[pl->last_g][3]));
    else
        HIP_TRY(hipStreamSynchronize(pl->last_stream));
    int64_t nnz = 0;
    int flags = 0;
    if (pl->P > 0) {
        // copies ordered behind the run on its own stream, waited for through
        // an event: neither the null stream nor other streams are involved
        HIP_TRY(hipMemcpyAsync(&nnz, pl->d_nnz + pl->P, sizeof(int64_t), hipMemcpyDeviceToHost, pl->last_stream));
        HIP_TRY(hipMemcpyAsync(&flags, pl->d_ints + kIntFlags, sizeof(int), hipMemcpyDeviceToHost, pl->last_stream));
        HIP_TRY(hipEventRecord(pl->copy_ev, pl->last_stream));
        HIP_TRY(hipEventSynchronize(pl->copy_ev));
    }
    pl->last_nnz = nnz;
    trace("sync: done nnz=%lld flags=%d", (long long)nnz, flags);
    if (flags & 4)
        return fail(QP_EINVAL, "a device sequence holds a residue code >= %d", alphabet_of(&pl->params));
    if (flags & 2)
        return fail(QP_EDEVICE, "a row held more entries above the threshold than its staging capacity");
    if ((flags & 1) || nnz > pl->pool_cap) {
        // the plan is left as it is: a caller makes a new plan with at least
        // this capacity (no buffer is replaced under captured graphs)
        if (res) {
            std::memset(res, 0, sizeof(*res));
            res->nnz = nnz;
        }
        return fail(QP_ENOSPC, "sparse output needed %lld entries, capacity %lld; create a plan with "
                    "nnz_capacity >= %lld", (long long)nnz, (long long)pl->pool_cap, (long long)nnz);
    }
    if (res) {
        res->n_pairs = pl->P;
        res->total_rows = pl->total_rows;
        res->nnz = nnz;
        res->pair_i = pl->d_pi;
        res->pair_j = pl->d_pj;
        res->row_off = pl->d_rowoff;
        res->row_ptr = pl->d_rowptr;
        res->nnz_off = pl->d_nnz;
        res->col = pl->d_col;
        res->val = pl->d_val;
        res->dist = pl->d_dist;
        res->log_z = pl->d_logz;
    }
    return QP_OK;
}

extern "C" qp_status qp_plan_download(qp_plan* pl, qp_result** out) { return qp::plan_download(pl, out, nullptr); }


qp_status qp_plan_timing(qp_plan* pl, double* kernel_ms, double* pipeline_ms, int64_t* n_runs, int32_t reset) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    HIP_TRY(hipSetDevice(pl->device));
    if (pl->ran && pl->last_g >= 0) HIP_TRY(hipEventSynchronize(pl->ev[pl->last_g][3]));
    collect_timing(pl);
    if (kernel_ms) *kernel_ms = pl->n_timed ? pl->sum_kernel_ms / pl->n_timed : 0.0;
    if (pipeline_ms) *pipeline_ms = pl->n_timed ? pl->sum_pipe_ms / pl->n_timed : 0.0;
    if (n_runs) *n_runs = pl->n_timed;
    if (reset) {
        pl->sum_kernel_ms = pl->sum_pipe_ms = 0.0;
        for (int c = 0; c < qp::kClasses; ++c) pl->sum_class_ms[c] = 0.0;
        pl->n_timed = 0;
    }
    return QP_OK;
}

qp_status qp_plan_class_timing(qp_plan* pl, int32_t cls, double* kernel_ms, int64_t* pairs, int64_t* cells,
                               int32_t* rows_per_lane) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    if (cls < 0 || cls >= qp::kClasses) return fail(QP_EINVAL, "class %d outside [0, %d)", cls, qp::kClasses);
    const qp_plan::ClassPlan& cp = pl->cls[cls];
    if (pairs) *pairs = cp.grid > 0 ? cp.pairs : 0;
    if (cells) *cells = cp.grid > 0 ? cp.cells : 0;
    if (rows_per_lane) *rows_per_lane = cp.grid > 0 ? cp.R : qp::class_rows_per_lane(cls);
    if (kernel_ms) {
        *kernel_ms = 0.0;
        if (cp.grid > 0 && pl->ran) {
            HIP_TRY(hipSetDevice(pl->device));
            if (pl->last_g >= 0) HIP_TRY(hipEventSynchronize(pl->ev[pl->last_g][3]));
            collect_timing(pl);
            *kernel_ms = pl->n_timed ? pl->sum_class_ms[cls] / pl->n_timed : 0.0;
        }
    }
    return QP_OK;
}

qp_status qp_plan_set_graph(qp_plan* pl, int32_t use_graph) {
    if (!pl) return fail(QP_EINVAL, "plan is NULL");
    pl->use_graph = use_graph != 0;
    return QP_OK;
}

int64_t qp_plan_device_bytes(const qp_plan* pl) { return pl ? pl->device_bytes : 0; }

void qp_plan_destroy(qp_plan* pl) {
    if (!pl) return;
    hipSetDevice(pl->device);
    if (pl->ran && pl->last_g >= 0) hipEventSynchronize(pl->ev[pl->last_g][3]);
    // nothing of a graph-launched plan may be in flight when its memory and
    // graphs go (eager runs are covered by the end event above)
    if (pl->ran && pl->exec[0]) (void)hipDeviceSynchronize();
    plan_free_device(pl);
    for (int g = 0; g < kNumEventSets; ++g) {
        for (int q = 0; q < 4; ++q)
            if (pl->ev[g][q]) hipEventDestroy(pl->ev[g][q]);
        for (int c = 0; c < qp::kClasses; ++c)
            for (int q = 0; q < 2; ++q)
                if (pl->cev[g][c][q]) hipEventDestroy(pl->cev[g][c][q]);
    }
    if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
    for (int q = 0; q < kMaxSide; ++q) {
        if (pl->side[q]) hipStreamDestroy(pl->side[q]);
        if (pl->join_ev[q]) hipEventDestroy(pl->join_ev[q]);
    }
    if (pl->fork_ev) hipEventDestroy(pl->fork_ev);
    if (pl->copy_ev) hipEventDestroy(pl->copy_ev);
    delete pl;
}

}  // extern "C"

// ------------------------------------------------- blocking host calls
static qp_status run_host(const uint8_t* const* seqs, const int32_t* lens, int32_t n, const int32_t* pi,
                          const int32_t* pj, int64_t np, const qp_params* params, float thresh, qp_result** out) {
    if (!out) return fail(QP_EINVAL, "out is NULL");
    *out = nullptr;
    qp_status st = validate_lens(lens, n);
    if (st != QP_OK) return st;
    if ((st = qp_params_check(params)) != QP_OK) return st;
    if (n > 0 && !seqs) return fail(QP_EINVAL, "seqs is NULL");
    for (int32_t i = 0; i < n; ++i) {
        if (!seqs[i]) return fail(QP_EINVAL, "seqs[%d] is NULL", i);
        for (int32_t c = 0; c < lens[i]; ++c)
            if (seqs[i][c] >= alphabet_of(params))
                return fail(QP_EINVAL, "seqs[%d][%d] = %d is not a residue code 0..%d", i, c, seqs[i][c],
                            alphabet_of(params) - 1);
    }
    if (!(thresh > 0.0f && thresh <= 1.0f)) return fail(QP_EINVAL, "thresh = %g is not in (0, 1]", (double)thresh);
    const int64_t P = pi ? np : (int64_t)n * (n - 1) / 2;
    if (pi && np < 0) return fail(QP_EINVAL, "n_pairs < 0");
    if (P == 0) {
        // nothing to compute: an empty result, without touching the device
        qp_result* r = qp::result_alloc(n, 0, 0, 0);
        if (!r) return fail(QP_ENOMEM, "out of host memory");
        r->thresh = thresh;
        *out = r;
        return QP_OK;
    }
    // Every plan is sized to the guaranteed output bound of its pairs, so no
    // run can overflow its sparse output and nothing is ever re-run.  When
    // the bound of the whole family does not fit a share of the free device
    // memory, the pairs are cut, in order, into chunks whose bounds do; the
    // chunks run one after the other and their results are concatenated.
    {
        int64_t bound = 0;  // validates the pair list before any device call
        if ((st = qp_output_bound(lens, n, pi, pj, np, thresh, &bound)) != QP_OK) return st;
    }
    int dev = 0;
    if ((st = check_device(&dev, nullptr)) != QP_OK) return st;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QP_EDEVICE, "hipMemGetInfo failed");
    }
    // pool and gathered output: 16 bytes per entry; a third of the free
    // memory leaves the rest to the per-wave workspace
    const int64_t max_entries = std::max<int64_t>(1, (int64_t)(free_b / 3) / 16);
    std::vector<int32_t> ci, cj;  // explicit pair list of every chunk
    std::vector<int64_t> cut{0};  // chunk k = pairs cut[k] .. cut[k+1]-1
    {
        try {
            ci.reserve((size_t)P);
            cj.reserve((size_t)P);
        } catch (const std::bad_alloc&) {
            return fail(QP_ENOMEM, "out of host memory");
        }
        int64_t acc = 0;
        auto add = [&](int32_t a, int32_t b) {
            const int64_t bp = (int64_t)lens[a] * row_bound(lens[b], thresh);
            if (acc > 0 && acc + bp > max_entries) {
                cut.push_back((int64_t)ci.size());
                acc = 0;
            }
            acc += bp;
            ci.push_back(a);
            cj.push_back(b);
        };
        if (pi) {
            for (int64_t k = 0; k < np; ++k) add(pi[k], pj[k]);
        } else {
            for (int32_t i = 0; i + 1 < n; ++i)
                for (int32_t j = i + 1; j < n; ++j) add(i, j);
        }
        cut.push_back(P);
    }
    const int n_chunks = (int)cut.size() - 1;
    trace("host: %lld pairs in %d chunk(s) of at most %lld bound entries", (long long)P, n_chunks,
          (long long)max_entries);
    std::vector<int64_t> off(std::max(n, 1));
    int64_t tot = 0;
    for (int32_t i = 0; i < n; ++i) {
        off[i] = tot;
        tot += lens[i];
    }
    uint8_t* h = nullptr;
    uint8_t* d = nullptr;
    int64_t* d_off = nullptr;
    hipStream_t s = nullptr;
    std::vector<qp_result*> parts((size_t)n_chunks, nullptr);
    auto cleanup = [&]() {
        if (s) hipStreamSynchronize(s);
        if (h) hipHostFree(h);
        if (d) hipFree(d);
        if (d_off) hipFree(d_off);
        if (s) hipStreamDestroy(s);
    };
    hipError_t e = hipHostMalloc((void**)&h, (size_t)std::max<int64_t>(tot, 1), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&d, (size_t)std::max<int64_t>(tot, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&d_off, sizeof(int64_t) * std::max(n, 1));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(QP_ENOMEM, "device staging allocation failed: %s", hipGetErrorString(e));
    }
    for (int32_t i = 0; i < n; ++i) std::memcpy(h + off[i], seqs[i], (size_t)lens[i]);
    e = hipMemcpyAsync(d, h, (size_t)std::max<int64_t>(tot, 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * std::max(n, 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cleanup();
        return fail(QP_EDEVICE, "host-to-device copy failed: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < n_chunks && st == QP_OK; ++k) {
        const int64_t c0 = cut[k], cn = cut[k + 1] - cut[k];
        qp_plan* pl = nullptr;
        // one chunk covering all pairs of an all-pairs family keeps the
        // implicit pair list
        const bool implicit = !pi && n_chunks == 1;
        st = qp_plan_create(lens, n, implicit ? nullptr : ci.data() + c0, implicit ? nullptr : cj.data() + c0,
                            implicit ? 0 : cn, params, thresh, -1, &pl);
        if (st == QP_OK) st = qp_plan_run(pl, d, d_off, s);
        if (st == QP_OK) st = qp_plan_download(pl, &parts[k]);
        if (pl) {
            std::string keep = g_err;
            qp_plan_destroy(pl);
            g_err = keep;
        }
    }
    std::string keep = g_err;
    cleanup();
    g_err = keep;
    if (st == QP_OK && n_chunks == 1) {
        *out = parts[0];
        parts[0] = nullptr;
    } else if (st == QP_OK) {
        // concatenate the chunks in pair order
        int64_t rows = 0, nnz = 0;
        for (qp_result* r : parts) {
            rows += r->total_rows;
            nnz += r->nnz;
        }
        qp_result* all = qp::result_alloc(n, P, rows, nnz);
        if (!all) {
            st = fail(QP_ENOMEM, "out of host memory for the concatenated result");
        } else {
            int64_t p0 = 0, r0 = 0, z0 = 0;
            double ms = 0.0;
            for (qp_result* r : parts) {
                const int64_t cp = r->n_pairs;
                std::memcpy(all->pair_i + p0, r->pair_i, sizeof(int32_t) * cp);
                std::memcpy(all->pair_j + p0, r->pair_j, sizeof(int32_t) * cp);
                for (int64_t q = 0; q < cp; ++q) {
                    all->row_off[p0 + q] = r0 + r->row_off[q];
                    all->nnz_off[p0 + q] = z0 + r->nnz_off[q];
                }
                std::memcpy(all->row_ptr + r0, r->row_ptr, sizeof(int32_t) * r->total_rows);
                std::memcpy(all->col + z0, r->col, sizeof(int32_t) * r->nnz);
                std::memcpy(all->val + z0, r->val, sizeof(float) * r->nnz);
                std::memcpy(all->dist + p0, r->dist, sizeof(double) * cp);
                std::memcpy(all->log_z + 2 * p0, r->log_z, sizeof(double) * 2 * cp);
                p0 += cp;
                r0 += r->total_rows;
                z0 += r->nnz;
                ms += r->device_ms;
            }
            all->row_off[P] = r0;
            all->nnz_off[P] = z0;
            all->device_ms = ms;
            all->thresh = thresh;
            *out = all;
        }
    }
    for (qp_result* r : parts) qp_result_free(r);
    return st;
}

extern "C" qp_status qp_posteriors(const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                                   const qp_params* params, float thresh, qp_result** out) {
    return run_host(seqs, lens, n, nullptr, nullptr, 0, params, thresh, out);
}

extern "C" qp_status qp_posteriors_pairs(const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                                         const int32_t* pair_i, const int32_t* pair_j, int64_t n_pairs,
                                         const qp_params* params, float thresh, qp_result** out) {
    if (!pair_i || !pair_j) {
        if (out) *out = nullptr;
        return fail(QP_EINVAL, "pair_i / pair_j are NULL");
    }
    return run_host(seqs, lens, n, pair_i, pair_j, n_pairs, params, thresh, out);
}
