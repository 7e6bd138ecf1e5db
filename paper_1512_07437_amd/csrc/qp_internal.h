// Internal interface between the C-ABI host code (qp_api.cpp) and the gfx950
// kernels (qp_device.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qp.h"

namespace qp {

constexpr int kWave = 64;           // lanes per wavefront on CDNA
constexpr int kWavesPerBlock = 4;   // one wave per SIMD of a CU
constexpr int kTabW = 32;           // stride of a table row (20 y codes, padded)
constexpr int kPadCode = 20;        // x code of rows past the end of a strip
constexpr int kTabRows = 21;        // 20 residues + the padding row
constexpr int kRMax = 8;            // largest rows-per-lane instantiation
constexpr int kMaxSeqLen = 1536;    // longest accepted sequence (QP_MAX_SEQ_LEN)
constexpr int kRescaleEvery = 8;    // steps between power-of-two rescales
constexpr int kKeyBins = 1024;      // queue keys: kernel class x cost bin
constexpr int kCostBins = 64;       // half-octave bins of m*n per kernel class
constexpr int kBandClass = kRMax;   // first banded class
constexpr int kBandRMin = 5;        // banded classes: 5..8 rows per lane
constexpr int kClasses = kBandClass + kRMax - kBandRMin + 1;  // 8 single band + 4 banded
constexpr int kTuneClasses = kBandClass + 1;  // tuning entries: 8 single band, one for all banded
static_assert(kClasses * kCostBins <= kKeyBins, "queue keys");

// Kernel class per minimal rows per lane: a pair whose row sequence needs
// r = ceil(m/64) <= 8 rows per lane runs in class c[r-1] (R = c+1 >= r rows
// per lane; the identity map uses the fewest), chosen per length bucket by
// the tuning table.  Longer rows are cut into nb = ceil(m / (64*8)) bands,
// each of 64 R rows with the fewest rows per lane R that still needs only nb
// bands (R = ceil(m / (64 nb)), 5..8 for m > 512): bands that fill their
// lanes, one banded class per R.
struct ClassMap {
    int8_t c[kRMax];
};
__host__ __device__ inline int banded_rows(int m) {
    const int nb = (m + kWave * kRMax - 1) / (kWave * kRMax);
    const int r = (m + kWave * nb - 1) / (kWave * nb);
    return r < kBandRMin ? kBandRMin : (r > kRMax ? kRMax : r);
}
__host__ __device__ inline int pair_class(int m, const ClassMap& map) {
    const int R = (m + kWave - 1) / kWave;
    return R <= kRMax ? map.c[R - 1] : kBandClass + banded_rows(m) - kBandRMin;
}
__host__ __device__ inline bool class_banded(int c) { return c >= kBandClass; }
__host__ __device__ inline int class_rows_per_lane(int c) { return c < kBandClass ? c + 1 : c - kBandClass + kBandRMin; }
// entry of the tuning arrays that applies to class c
__host__ __device__ inline int tune_index(int c) { return c < kBandClass ? c : kBandClass; }

// Model constants in the scaled-variable form used by the kernels, computed
// on the device from the raw parameters (k_tables).
struct DevConsts {
    double tau;        // M->M of the pair-HMM
    double eps1, eps2; // gap extension per class
    double c1, c2;     // delta_k * (1 - eps_k)
    double u, o;       // partition function: extension and opening weights
    double w_hmm;      // weight of the HMM posterior
};

// Raw parameters as copied to the device for k_tables.
struct DevParams {
    double joint[400];
    double score[400];
    double gap_open[2];
    double gap_extend[2];
    double pf_gap_open, pf_gap_extend, temperature, w_hmm;
    int32_t n_gap_classes;
    int32_t alphabet;  // residue codes 0..alphabet-1
};

struct PairArgs {
    // inputs
    const uint8_t* seqs;
    const int64_t* seq_off;
    const int32_t* lens;
    const int32_t* pair_i;
    const int32_t* pair_j;
    const int32_t* queue;       // pair ids in processing order (class-major)
    const uint8_t* tr;          // per pair: 1 = swept with the second sequence as rows (null: none)
    int64_t n_pairs;
    int* queue_head;            // [kClasses] per-class queue heads
    const int* hist;            // [kKeyBins] pairs per queue key
    const int* bin_start;       // [kKeyBins] first queue slot of each key
    int cls;                    // kernel class this launch serves
    const void* tab;            // [kTabRows * kTabW] (e_hmm, w_pf) pairs
    const void* col0;           // per row: D(i,0) of both models
    const DevConsts* consts;
    float thresh;
    int cap;                    // staging entries per row (the class's widest rows)
    int cap_thresh;             // floor(1 / thresh) + 1, at most kMaxSeqLen + 1: entries per output row of
                                // a transposed pair are at most min(its rows, cap_thresh)
    // outputs
    const int64_t* row_off;
    int32_t* row_ptr;
    int64_t* pair_nnz;          // [n_pairs + 1]
    int64_t* pair_base;         // [n_pairs]
    int32_t* pool_col;
    float* pool_val;
    int64_t pool_cap;
    unsigned long long* pool_head;
    double* dist;
    double* logz;
    int* flags;                 // bit0 pool overflow, bit1 staging overflow
    // per-wave scratch slots
    char* scratch;
    int64_t slot_bytes;
    int64_t off_exps, off_fb, off_bb, off_log;
    int64_t spill_band_stride;  // value pairs per band
    int64_t exps_band_stride;   // int2 per band
    int64_t bnd_stride;         // boundary records per buffer
};

// kernels launched by the host code (qp_device.hip)
// copies each sequence to a 4-byte aligned slot of seqa (zero padded) and
// sets bit 4 of *flags if a code is outside 0..19
hipError_t launch_stage_seqs(int32_t n, int32_t alphabet, const uint8_t* seqs, const int64_t* seq_off, const int32_t* lens,
                             const int64_t* seqa_off, uint8_t* seqa, int* flags, hipStream_t s);
hipError_t launch_tables(const DevParams* p, void* tab, DevConsts* c, void* col0, int rows, int fp64,
                         hipStream_t s);
size_t col0_bytes();
hipError_t launch_reset(int* ints, int n_ints, hipStream_t s);
hipError_t launch_setup(int32_t n, const int32_t* lens, const int32_t* list_i, const int32_t* list_j,
                        const uint8_t* tr, int64_t n_pairs, int32_t* pair_i, int32_t* pair_j, int64_t* rows1,
                        int32_t* key, int* hist, int64_t* pair_nnz, const ClassMap& map, hipStream_t s);
hipError_t launch_bins(const int* hist, int* bin_start, hipStream_t s);
hipError_t launch_fill_queue(int64_t n_pairs, const int32_t* key, const int* bin_start, int* bin_fill,
                             int32_t* queue, hipStream_t s);
// exclusive scan of n int64 values in place; tmp must hold scan_tmp_elems(n)
int64_t scan_tmp_elems(int64_t n);
hipError_t scan_i64(int64_t* data, int64_t n, int64_t* tmp, hipStream_t s);
hipError_t launch_pairs(int cls, int fp64, int grid, const PairArgs& a, hipStream_t s);
// the plain per-pair form: pair p alone, one wave, scratch slot 0 of a.scratch
hipError_t launch_pair_one(int cls, int fp64, int64_t p, const PairArgs& a, hipStream_t s);
int pairs_blocks_per_cu(int cls, int fp64);
// checkpointed FP32 form of the pair kernels (forward values recomputed per
// block in the backward sweep instead of spilled); a slot holds, per band,
// the saved forward state of every block (ck_state_words(R) words per lane)
// in place of the spilled values and exponents, and the forward boundary
// records of every band
constexpr int kCkMaxClass = 4;  // single-band classes 0..4 (1..5 rows per lane) have the form,
constexpr int kCkBandRows = 4;  // and the banded class, in bands of 64 * 4 rows
// rows per lane a class runs with in a given form
inline int class_rows(int c, bool ck) { return ck && class_banded(c) ? kCkBandRows : class_rows_per_lane(c); }
hipError_t launch_pairs_ck(int cls, int grid, const PairArgs& a, hipStream_t s);
hipError_t launch_pair_one_ck(int cls, int64_t p, const PairArgs& a, hipStream_t s);
int pairs_ck_blocks_per_cu(int cls);
int ck_state_words(int R);
hipError_t launch_gather(int64_t n_pairs, const int64_t* nnz_off, const int64_t* pair_base, const int32_t* pool_col, const float* pool_val,
                         int32_t* col, float* val, int64_t cap, hipStream_t s);
size_t fwd_bnd_bytes(int fp64);
size_t bwd_bnd_bytes(int fp64);

// plan building blocks shared with the serving loop (qp_api.cpp)
qp_status plan_shape(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j, int64_t n_pairs,
                     const qp_params* params, float thresh, int64_t nnz_capacity, int64_t wave_budget,
                     qp_plan** plan);
int64_t plan_bytes(qp_plan* pl);
// sparse entries produced by the plan's last synchronised run
int64_t plan_last_nnz(const qp_plan* pl);
// Optional device allocator of a plan, set before plan_materialize: the
// serving loop keeps freed blocks for the next family instead of handing
// them back to the runtime between families.
struct DeviceAllocator {
    void* (*alloc)(void* ctx, size_t bytes);  // nullptr when it cannot
    void (*release)(void* ctx, void* p);
    void* ctx;
};
void plan_set_allocator(qp_plan* pl, const DeviceAllocator& a);
// run every kernel class on the run stream (no forked side streams)
void plan_set_single_stream(qp_plan* pl, bool on);
// Pinned staging for downloads: results are copied in chunks of `half`
// bytes through the two halves of `buf`, the copy of one half overlapping
// the host copy out of the other.  Owned by the caller.
struct Staging {
    char* buf = nullptr;
    size_t half = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
// qp_plan_download; results in pageable memory go through the staging
// buffer when one is given
qp_status plan_download(qp_plan* pl, qp_result** out, Staging* stg);
// A result with room for the given counts (every array at least one element;
// row_off[0] = nnz_off[0] = 0), in one host block that is pinned where that
// pays off; nullptr when out of host memory.  Freed by qp_result_free.
qp_result* result_alloc(int32_t n_seqs, int64_t P, int64_t rows, int64_t nnz);
// whether the result's arrays are in pinned memory
bool result_pinned(const qp_result* r);
qp_status plan_materialize(qp_plan* pl);
qp_status set_error(qp_status st, const char* msg);
// formatted error message for qp_last_error; returns st
qp_status fail_msg(qp_status st, const char* fmt, ...);

// host helpers shared by the entry points (qp_api.cpp)
int alphabet_of(const qp_params* p);               // residue codes 0..alphabet-1
int64_t row_bound(int32_t cols, float thresh);     // slots of one output row
qp_status validate_lens(const int32_t* lens, int32_t n);
qp_status check_device(int* dev, int* n_cu);       // current device is gfx950
void current_tuning(ClassMap* map, double* waves_frac, int* recompute);  // the tuning table in force
// layout of one per-wave scratch slot of a kernel class with R rows per lane,
// at most mmax rows, nmax columns and nb_max bands, cap output slots per row;
// ck: the checkpointed form's layout
void slot_layout(int R, int mmax, int nmax, int nb_max, int cap, int fp64, bool ck, PairArgs* a);

}  // namespace qp
