// gfx950 kernels of the all-pairs posterior engine (stage I of QuickProbs 2:
// posterior matrices of every pair from a pair-HMM and a partition function,
// Methods, opening paragraph; sparse storage, "Selective consistency"
// footnote; maximum-expected-accuracy scores for the distances).
//
// Layout of one pair on one wavefront
// -----------------------------------
// Rows (residues of x) are striped over the 64 lanes: lane l owns rows
// l*R .. l*R+R-1 of a band of 64*R rows; an x longer than 512 is cut into
// ceil(m/512) bands of R = ceil(m / (64 * bands)) rows per lane, processed
// one after the other (each R its own kernel class).  x is the pair's first
// sequence, or its second when the host finds the transposed sweep cheaper
// (the models are symmetric, so P(y, x) = P(x, y)^T; such a pair's output
// rows are the sweep's columns).  Columns (residues of y) are swept in a skewed
// wavefront: at step s lane l handles column j = s - l + 1, so the row above
// its strip (lane l-1) finished column j one step earlier and hands its last
// row over with one DPP wave shift.  The backward pass runs the same skew in
// the opposite direction (lane l+1 leads).
//
// Numbers.  Values are FP32 (or FP64) with a power-of-two scale per lane and
// model: the stored value is true * 2^-E.  Values received from a neighbour
// are re-based with ldexp, all lanes rescale together every kRescaleEvery
// steps, and exponents are exact integers, so Z and the posteriors carry no
// rounding from the scaling itself.
//
// Posteriors need the forward match value at the same cell as the backward
// one.  The spilling form stores (f_hmm, f_pf) per cell, step-major and lane-
// contiguous, so both the store and the reversed read are fully coalesced;
// the checkpointed form saves the forward state every 8 steps and recomputes
// each block in registers during the backward sweep.  The backward pass
// fuses the posterior, the average of the two models, the threshold, the
// hit log of CSR entries and the reverse MEA recursion.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "qp_internal.h"
#include "qp_wave.h"

namespace qp {

template <typename T> struct Pair2;
template <> struct Pair2<float> { using type = float2; };
template <> struct Pair2<double> { using type = double2; };

// forward boundary record: last row of a band at one column
template <typename T> struct FwdBnd {
    T M, U1, U2, D, gM, gU, gD;
    int EH, EP;
};
// backward boundary record: first row of a band at one column
template <typename T> struct BwdBnd {
    T U1, U2, Tt, gU, gT;
    double A;
    int FH, FP;
};

// Spill traffic is written once and read back once, long after any cache
// could keep it: streaming (non-temporal) stores and loads, so it does not
// displace other lines from L2 and the last-level cache.
template <typename V2>
__device__ __forceinline__ void spill_store(V2* p, const V2& v) {
    using S = decltype(v.x);
    typedef S N2 __attribute__((ext_vector_type(2)));
    const N2 n = {v.x, v.y};
    __builtin_nontemporal_store(n, reinterpret_cast<N2*>(p));
}
template <typename V2>
__device__ __forceinline__ V2 spill_load(const V2* p) {
    using S = decltype(p->x);
    typedef S N2 __attribute__((ext_vector_type(2)));
    const N2 n = __builtin_nontemporal_load(reinterpret_cast<const N2*>(p));
    V2 v;
    v.x = n[0];
    v.y = n[1];
    return v;
}

template <typename T> struct Coef {
    T tau, eps1, eps2, c1, c2, u, o;
};

// D(i,0) of both models for row i (1-based, index i-1): mantissa and exponent
struct Col0 {
    double mH, mP;
    int eH, eP;
};

// ---------------------------------------------------------------- helpers
constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l-1
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l+1

template <int CTRL> __device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
    long long b = __double_as_longlong(v);
    int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL));
    int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float qldexp(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
__device__ __forceinline__ double qldexp(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ __forceinline__ int qexp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ int qexp(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ float qmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double qmax(double a, double b) { return fmax(a, b); }

// 2^(e*lg - sh) with 0^0 = 1 (lg = log2 of a base that may be 0)
__device__ __forceinline__ double pow2s(double lg, int e, int sh) {
    return e == 0 ? exp2(-(double)sh) : exp2((double)e * lg - (double)sh);
}


__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Residue idx of a sequence whose copy is 4-byte aligned and zero padded to
// a multiple of 4 bytes: a uniform index makes this a scalar (SMEM) load, so
// the step loops issue no vector loads for y and never wait on their stores.
__device__ __forceinline__ int res_uniform(const uint8_t* y, int idx) {
    typedef __attribute__((address_space(4))) const uint32_t cu32;
    const uint64_t a = (uint64_t)(uintptr_t)y;
    const cu32* w = (const cu32*)(uintptr_t)a;
    return (int)((w[idx >> 2] >> ((idx & 3) * 8)) & 0xffu);
}

// Band position modes of the band routines: 1 / 0 fix "top band" (or
// "bottom band") at compile time, so single-band pairs carry no boundary
// code; kBandRuntime takes it from a wave-uniform flag (scalar branches).
constexpr int kBandRuntime = 2;
__device__ __forceinline__ bool band_is(int mode, bool rt) { return mode == kBandRuntime ? rt : mode == 1; }

// ---------------------------------------------------------------- forward
// One band of rows [r0, r0+rows) of pair (x, y); L lanes carry R rows each.
template <int R, typename T, int FM, int LM>
__device__ void fwd_band(int lane, const uint8_t* __restrict__ x, const uint8_t* __restrict__ y, int n, int r0,
                         int rows, int L, const typename Pair2<T>::type* tab,
                         const Coef<T>& k, const Col0* __restrict__ col0,
                         typename Pair2<T>::type* __restrict__ spill, int2* __restrict__ exps,
                         const FwdBnd<T>* __restrict__ fin, FwdBnd<T>* __restrict__ fout, T& zH, T& zP,
                         int& ezH, int& ezP, bool rt_first, bool rt_last) {
    using V2 = typename Pair2<T>::type;
    const bool first = band_is(FM, rt_first), last = band_is(LM, rt_last);
    const bool used = lane < L;
    int xo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int row = lane * R + r;
        xo[r] = (used && row < rows ? (int)x[r0 + row] : kPadCode) * kTabW;
    }
    // carried per row: W_k = V_k at the lane's next column (horizontal gap
    // runs, already extended by this column's match), D = into-M sum of the
    // current column (the diagonal input of the row below); PF alike
    T W1[R], W2[R], D[R], gW[R], gD[R];
    int EH, EP;
    {
        // column 0: only vertical gap runs from the virtual begin state,
        // D(i,0) = sum_k c_k eps_k^(i-1) (PF: o u^(i-1)), tabulated per row
        Col0 c0[R];
        EH = INT_MIN;
        EP = INT_MIN;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = lane * R + r;  // rows past the band are padding: zero
            if (used && row < rows) {
                c0[r] = col0[r0 + row];
            } else {
                c0[r].mH = 0.0;
                c0[r].mP = 0.0;
                c0[r].eH = 0;
                c0[r].eP = 0;
            }
            EH = max(EH, c0[r].mH != 0.0 ? c0[r].eH : INT_MIN);
            EP = max(EP, c0[r].mP != 0.0 ? c0[r].eP : INT_MIN);
        }
        if (EH == INT_MIN) EH = 0;
        if (EP == INT_MIN) EP = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            W1[r] = T(0);  // V_k(i,1) = M(i,0) + eps V_k(i,0) = 0
            W2[r] = T(0);
            gW[r] = T(0);
            D[r] = qldexp((T)c0[r].mH, c0[r].eH - EH);
            gD[r] = qldexp((T)c0[r].mP, c0[r].eP - EP);
        }
    }
    // vertical values of the strip's last row at the lane's current column,
    // handed to the lane below together with D[R-1], gD[R-1] and EH, EP
    T oM = T(0), oU1 = T(0), oU2 = T(0), ogM = T(0), ogU = T(0);
    // diagonal input of the strip's first row (row above, previous column)
    T aD = T(0), gaD = T(0);
    // virtual row 0 (first band, lane 0): V_k(0,j) = eps_k^(j-1), j >= 1
    T tv1 = T(0), tv2 = T(0), tgv = T(0);
    if (lane == 0) {
        if (first) {
            aD = qldexp(k.tau, -EH);     // D(0,0): the begin state
            gaD = qldexp(T(1), -EP);
            tv1 = qldexp(T(1), -EH);
            tv2 = tv1;
            tgv = qldexp(T(1), -EP);
        } else {
            const FwdBnd<T> b = fin[0];
            aD = qldexp(b.D, b.EH - EH);
            gaD = qldexp(b.gD, b.EP - EP);
        }
    }
    if (!last && lane == L - 1) {
        FwdBnd<T> b;
        b.M = T(0); b.U1 = T(0); b.U2 = T(0); b.D = D[R - 1];
        b.gM = T(0); b.gU = T(0); b.gD = gD[R - 1];
        b.EH = EH; b.EP = EP;
        fout[0] = b;
    }

    const int S = n + L - 1;
    // residue of the lane's column: lane 0 reads y[s] (scalar), lane l takes
    // lane l-1's residue of the previous step
    int ycur = 0;
    int y0n = res_uniform(y, 0);
    FwdBnd<T> bq;  // lane 0 of a lower band: boundary record of its next column
    if (!first && lane == 0) bq = fin[1];
    // spill values of the current step; lanes outside their columns store
    // stale values, so every store covers whole cache lines (a partial line
    // costs a read-modify-write in HBM) and nothing reads them back
    V2 sm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { sm[r].x = T(0); sm[r].y = T(0); }
    auto fstep = [&](const int s) {
        const int j = s - lane + 1;
        const bool active = used && j >= 1 && j <= n;
        {
            const int y0 = y0n;
            y0n = res_uniform(y, min(s + 1, n - 1));
            const int yup = dpp_i<kDppWaveShr1>(ycur);
            ycur = lane == 0 ? y0 : yup;
        }
        // ---- exchange with the lane above
        T rM = dpp<kDppWaveShr1>(oM), rU1 = dpp<kDppWaveShr1>(oU1), rU2 = dpp<kDppWaveShr1>(oU2);
        T rD = dpp<kDppWaveShr1>(D[R - 1]), rgM = dpp<kDppWaveShr1>(ogM), rgU = dpp<kDppWaveShr1>(ogU);
        T rgD = dpp<kDppWaveShr1>(gD[R - 1]);
        int rEH = dpp_i<kDppWaveShr1>(EH), rEP = dpp_i<kDppWaveShr1>(EP);
        if (lane == 0) {
            if (first) {
                rM = T(0); rU1 = T(0); rU2 = T(0);
                rD = k.c1 * tv1 + k.c2 * tv2;
                rgM = T(0); rgU = T(0);
                rgD = k.o * tgv;
                rEH = EH; rEP = EP;
                tv1 *= k.eps1; tv2 *= k.eps2; tgv *= k.u;
            } else {
                rM = bq.M; rU1 = bq.U1; rU2 = bq.U2; rD = bq.D;
                rgM = bq.gM; rgU = bq.gU; rgD = bq.gD;
                rEH = bq.EH; rEP = bq.EP;
                bq = fin[s + 2 <= n ? s + 2 : n];
            }
        }
        {
            const int dH = rEH - EH, dP = rEP - EP;
            rM = qldexp(rM, dH); rU1 = qldexp(rU1, dH); rU2 = qldexp(rU2, dH); rD = qldexp(rD, dH);
            rgM = qldexp(rgM, dP); rgU = qldexp(rgU, dP); rgD = qldexp(rgD, dP);
        }
        // match terms of every row first, for all lanes: row r's diagonal
        // input is row r-1's into-M sum of the previous column (the lane
        // above's for row 0).  Lanes outside their columns compute values
        // nobody reads (they go to the spill as stale lines only).  With the
        // old sums consumed here, the sums of this column overwrite them in
        // place below.
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V2 e = tab[xo[r] + ycur];
            sm[r].x = e.x * (r == 0 ? aD : D[r - 1]);
            sm[r].y = e.y * (r == 0 ? gaD : gD[r - 1]);
        }
        oM = sm[R - 1].x;
        ogM = sm[R - 1].y;
        if (active) {
            T upM = rM, upU1 = rU1, upU2 = rU2;
            T gupM = rgM, gupU = rgU;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T nM = sm[r].x, ngM = sm[r].y;
                const T nU1 = fma(k.eps1, upU1, upM);
                const T nU2 = fma(k.eps2, upU2, upM);
                D[r] = fma(k.c2, nU2 + W2[r], fma(k.c1, nU1 + W1[r], k.tau * nM));
                const T ngU = fma(k.u, gupU, gupM);
                gD[r] = fma(k.o, ngU + gW[r], ngM);
                W1[r] = fma(k.eps1, W1[r], nM);
                W2[r] = fma(k.eps2, W2[r], nM);
                gW[r] = fma(k.u, gW[r], ngM);
                upM = nM; upU1 = nU1; upU2 = nU2;
                gupM = ngM; gupU = ngU;
            }
            oU1 = upU1; oU2 = upU2;
            ogU = gupU;
            if (!last && lane == L - 1) {
                FwdBnd<T> b;
                b.M = oM; b.U1 = oU1; b.U2 = oU2; b.D = D[R - 1];
                b.gM = ogM; b.gU = ogU; b.gD = gD[R - 1];
                b.EH = EH; b.EP = EP;
                fout[j] = b;
            }
        }
        {
            V2* sp = spill + (int64_t)s * R * kWave;  // uniform step base
#pragma unroll
            for (int r = 0; r < R; ++r) spill_store(&sp[r * kWave + lane], sm[r]);
        }
        // exponents change only at the rescale closing every block of
        // kRescaleEvery steps: one record per block, written by every lane
        if ((s % kRescaleEvery) == 0) (exps + (int64_t)(s / kRescaleEvery) * kWave)[lane] = make_int2(EH, EP);
        aD = rD;
        gaD = rgD;
    };
    // power-of-two rescale closing every block of kRescaleEvery steps (a
    // separate call after each whole block, so that the step loop carries
    // one set of registers)
    auto rescale = [&]() {
        {
            T mh = T(0), mp = T(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                mh = qmax(mh, D[r]);
                mp = qmax(mp, gD[r]);
            }
            const int sh = -qexp(mh), sp = -qexp(mp);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                W1[r] = qldexp(W1[r], sh); W2[r] = qldexp(W2[r], sh); D[r] = qldexp(D[r], sh);
                gW[r] = qldexp(gW[r], sp); gD[r] = qldexp(gD[r], sp);
            }
            oM = qldexp(oM, sh); oU1 = qldexp(oU1, sh); oU2 = qldexp(oU2, sh);
            aD = qldexp(aD, sh); tv1 = qldexp(tv1, sh); tv2 = qldexp(tv2, sh);
            ogM = qldexp(ogM, sp); ogU = qldexp(ogU, sp);
            gaD = qldexp(gaD, sp); tgv = qldexp(tgv, sp);
            EH -= sh;
            EP -= sp;
        }
    };
    int s0 = 0;
    for (; s0 + kRescaleEvery <= S; s0 += kRescaleEvery) {
        for (int q = 0; q < kRescaleEvery; ++q) fstep(s0 + q);
        rescale();
    }
    for (; s0 < S; ++s0) fstep(s0);
    if (last) {
        // Z = D(m, n): last real row of the band, held by lane L-1
        const int rm = (rows - 1) - (L - 1) * R;
        T zd = T(0), zg = T(0);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r == rm) { zd = D[r]; zg = gD[r]; }
        zH = rdlane(zd, L - 1);
        zP = rdlane(zg, L - 1);
        ezH = rdlane(EH, L - 1);
        ezP = rdlane(EP, L - 1);
    }
}

// Hit log of one backward step: the rows of hbits hit at column j.  Each
// record is (output row, rank from the output row's end, output column,
// value); the wave appends its records as one contiguous run per row index.
// Normal pair: output row = the row, rank = its hits so far (cnt, already
// counting this one), columns met in decreasing order.  Transposed pair
// (swept with the second sequence as rows): output row = the column j-1,
// output column = the row; a column meets its rows in decreasing order, the
// lane's rows at this step last (highest row first), so a row's rank is the
// column's hits before this step (one LDS atomic per lane adds them all)
// plus the lane's hit rows above it.  Hits past a row's capacity are counted
// but not logged.  The log holds log_cap records; a pair whose hits would
// pass that (not possible for posteriors: at most min(m, n) / thresh of them
// reach the threshold) stops logging and is reported (flag bit 1).
template <int R>
__device__ __forceinline__ void log_hits(int hbits, bool trp, int* __restrict__ colcnt, const int (&cnt)[R],
                                         int cap, int j, int r0, int lane, const float (&pv)[R],
                                         int4* __restrict__ hitlog, int& nlog, int log_cap, int* __restrict__ flags) {
    if (!__ballot(hbits != 0)) return;
    int old = 0;
    if (trp && hbits != 0) old = atomicAdd(&colcnt[j - 1], __popc((unsigned)hbits));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool h = ((hbits >> r) & 1) != 0;
        const int rk = trp ? old + __popc((unsigned)hbits >> (r + 1)) : cnt[r] - 1;
        const bool keep = h && rk < cap;
        const unsigned long long km = __ballot(keep);
        if (km) {
            const int rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0));
            const int row = r0 + lane * R + r;
            if (keep && nlog + rank < log_cap)
                hitlog[nlog + rank] = make_int4(trp ? j - 1 : row, rk, trp ? row : j - 1, __float_as_int(pv[r]));
            const int nn = nlog + __popcll(km);
            if (nn > log_cap && lane == 0) atomicOr(flags, 2);
            nlog = __builtin_amdgcn_readfirstlane(min(nn, log_cap));
        }
    }
}

// --------------------------------------------------------------- backward
// FIRST / LAST: the band is the top / bottom band of the pair (band position
// modes as in the forward routine).
template <int R, typename T, int FM, int LM>
__device__ void bwd_band(int lane, const uint8_t* __restrict__ x, const uint8_t* __restrict__ y, int n, int r0,
                         int rows, int L, const typename Pair2<T>::type* tab, const Coef<T>& k,
                         const typename Pair2<T>::type* __restrict__ spill, const int2* __restrict__ exps,
                         const BwdBnd<T>* __restrict__ bin, BwdBnd<T>* __restrict__ bout, T invZH, T invZP, int ezH,
                         int ezP, float thresh, int cap, int4* __restrict__ hitlog, int& nlog,
                         int32_t* __restrict__ rowcnt, int* __restrict__ flags,
                         double& a11, bool rt_first, bool rt_last, bool trp, int* __restrict__ colcnt,
                         int log_cap) {
    using V2 = typename Pair2<T>::type;
    const bool FIRST = band_is(FM, rt_first), LAST = band_is(LM, rt_last);
    const bool used = lane < L;
    int xo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int row = lane * R + r;
        xo[r] = (used && row < rows ? (int)x[r0 + row] : kPadCode) * kTabW;
    }
    // carried per row (values at column j+1): bV1, bV2 (horizontal),
    // Tp = e * bM (diagonal input of the row above), A (reverse MEA)
    T bV1[R], bV2[R], Tp[R], gbV[R], gTp[R];
    double A[R];
    int cnt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bV1[r] = T(0); bV2[r] = T(0); Tp[r] = T(0); gbV[r] = T(0); gTp[r] = T(0);
        A[r] = 0.0;
        cnt[r] = 0;
    }
    int FH = 0, FP = 0;
    // diagonal input of the strip's last row (row below, next column)
    T bT = T(0), bgT = T(0);
    double bA = 0.0;
    if (LAST && lane == L - 1) {
        // end state: the cell after (m, n) contributes weight w/Z to (m, n);
        // every backward value is then already divided by Z (mantissa) and
        // weighted, so the posterior is f * b times a power of two
        const int rm = (rows - 1) - (L - 1) * R;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r == rm + 1) { Tp[r] = invZH; gTp[r] = invZP; }
        if (rm + 1 == R) { bT = invZH; bgT = invZP; }
    }
    // vertical values of the strip's first row at the lane's current column,
    // handed to the lane above together with Tp[0], gTp[0], A[0] and FH, FP
    T oU1 = T(0), oU2 = T(0), ogU = T(0);

    const int S = n + L - 1;
    const int lead = L - 1 - lane;  // lane L-1 starts at column n
    // residue of the lane's column: lane L-1 reads y[n-1-t] (scalar), lane l
    // takes lane l+1's residue of the previous step
    int ycur = 0;
    int yLn = res_uniform(y, n - 1);
    V2 fa[R], fb[R];
    int2 ea = make_int2(0, 0), eb = make_int2(0, 0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        fa[r].x = T(0); fa[r].y = T(0); fb[r].x = T(0); fb[r].y = T(0);
    }
    if (used && lead == 0) {
        const V2* sp = spill + (int64_t)(S - 1) * R * kWave;
#pragma unroll
        for (int r = 0; r < R; ++r) fa[r] = spill_load(&sp[r * kWave + lane]);
        ea = (exps + (int64_t)((S - 1) / kRescaleEvery) * kWave)[lane];
    }
    BwdBnd<T> bq;  // lane L-1 of an upper band: boundary record of its next column
    if (!LAST && lane == L - 1) bq = bin[n];

    // one step: uses the forward values in fc/ec, prefetches the next step's
    // into fn/en
    auto step = [&](const int t, const V2 (&fc)[R], const int2 ec, V2 (&fn)[R], int2& en) {
        const int j = n - t + lead;
        const bool active = used && j >= 1 && j <= n;
        // prefetch the next step unconditionally (clamped in range), so the
        // loads are straight-line and the wait for them is counted exactly;
        // lanes outside their columns never read what they loaded
        const int tn = t + 1 < S ? S - 2 - t : 0;
        {
            const int yl = yLn;
            yLn = res_uniform(y, max(n - t - 2, 0));
            const int ydn = dpp_i<kDppWaveShl1>(ycur);
            ycur = lane == L - 1 ? yl : ydn;
        }
        {
            const V2* sp = spill + (int64_t)tn * R * kWave;
#pragma unroll
            for (int r = 0; r < R; ++r) fn[r] = spill_load(&sp[r * kWave + lane]);
            en = (exps + (int64_t)(tn / kRescaleEvery) * kWave)[lane];
        }
        // ---- exchange with the lane below
        T rU1 = dpp<kDppWaveShl1>(oU1), rU2 = dpp<kDppWaveShl1>(oU2), rT = dpp<kDppWaveShl1>(Tp[0]);
        T rgU = dpp<kDppWaveShl1>(ogU), rgT = dpp<kDppWaveShl1>(gTp[0]);
        double rA = dpp<kDppWaveShl1>(A[0]);
        int rFH = dpp_i<kDppWaveShl1>(FH), rFP = dpp_i<kDppWaveShl1>(FP);
        const bool edge = lane == L - 1;
        if (LAST) {
            // below the last row: nothing (the end state entered via bT/Tp)
            rU1 = edge ? T(0) : rU1;
            rU2 = edge ? T(0) : rU2;
            rT = edge ? T(0) : rT;
            rgU = edge ? T(0) : rgU;
            rgT = edge ? T(0) : rgT;
            rA = edge ? 0.0 : rA;
            rFH = edge ? FH : rFH;
            rFP = edge ? FP : rFP;
        } else {
            rU1 = edge ? bq.U1 : rU1;
            rU2 = edge ? bq.U2 : rU2;
            rT = edge ? bq.Tt : rT;
            rgU = edge ? bq.gU : rgU;
            rgT = edge ? bq.gT : rgT;
            rA = edge ? bq.A : rA;
            rFH = edge ? bq.FH : rFH;
            rFP = edge ? bq.FP : rFP;
            if (edge) bq = bin[j - 1 >= 1 ? j - 1 : 1];
        }
        {
            // A lane that has not started yet (and the first step of it)
            // holds no state except the diagonal input; it takes over the
            // exponent of the values flowing in, so that nothing is converted
            // across a large exponent gap (right-edge values far above the
            // last row are ~eps^(m-i) and would underflow in FP32).  The lane
            // holding the end state keeps its own scale.
            const bool adopt = j >= n && !(LAST && lane == L - 1);
            const int nFH = adopt ? rFH : FH, nFP = adopt ? rFP : FP;
            bT = qldexp(bT, FH - nFH);
            bgT = qldexp(bgT, FP - nFP);
            FH = nFH;
            FP = nFP;
            const int dH = rFH - FH, dP = rFP - FP;
            rU1 = qldexp(rU1, dH); rU2 = qldexp(rU2, dH); rT = qldexp(rT, dH);
            rgU = qldexp(rgU, dP); rgT = qldexp(rgT, dP);
        }
        int hbits = 0;  // rows of this step at or above the threshold
        float pv[R];    // and their posteriors
        if (active) {
            T dU1 = rU1, dU2 = rU2, dgU = rgU;
            double dA = rA;
            T dgT = bT, dggT = bgT;
            double dgA = bA;
            const int kH = ec.x + FH - ezH, kP = ec.y + FP - ezP;
#pragma unroll
            for (int r = R - 1; r >= 0; --r) {
                const V2 e = tab[xo[r] + ycur];
                const T t1 = dgT, tg = dggT;
                const T nU1 = fma(k.eps1, dU1, t1);
                const T nU2 = fma(k.eps2, dU2, t1);
                const T nV1 = fma(k.eps1, bV1[r], t1);
                const T nV2 = fma(k.eps2, bV2[r], t1);
                const T bM = fma(k.c2, dU2 + bV2[r], fma(k.c1, dU1 + bV1[r], k.tau * t1));
                const T nT = e.x * bM;
                const T ngU = fma(k.u, dgU, tg);
                const T ngV = fma(k.u, gbV[r], tg);
                const T gbM = fma(k.o, dgU + gbV[r], tg);
                const T ngT = e.y * gbM;
                const T pH = qldexp(fc[r].x * bM, kH);
                const T pP = qldexp(fc[r].y * gbM, kP);
                const T P = pH + pP;
                const double nA = fmax(dgA + (double)P, fmax(dA, A[r]));
                const int row = lane * R + r;
                const bool hit = P >= (T)thresh && row < rows;
                pv[r] = (float)P;
                hbits |= hit ? (1 << r) : 0;
                cnt[r] += hit ? 1 : 0;
                dgT = Tp[r]; dggT = gTp[r]; dgA = A[r];
                Tp[r] = nT; gTp[r] = ngT; A[r] = nA;
                bV1[r] = nV1; bV2[r] = nV2; gbV[r] = ngV;
                dU1 = nU1; dU2 = nU2; dgU = ngU; dA = nA;
            }
            oU1 = dU1; oU2 = dU2; ogU = dgU;
            if (!FIRST && lane == 0) {
                BwdBnd<T> b;
                b.U1 = oU1; b.U2 = oU2; b.Tt = Tp[0]; b.gU = ogU; b.gT = gTp[0]; b.A = A[0];
                b.FH = FH; b.FP = FP;
                bout[j] = b;
            }
        }
        // append this step's hits to the hit log, one contiguous run per row
        // index across the wave (whole lines fill up in cache instead of
        // sparse 4-byte writes); record = (row, rank from the row's end,
        // column, value).  Uniform control flow keeps the log position in a
        // scalar; a row past its capacity keeps counting and is reported.
        log_hits<R>(hbits, trp, colcnt, cnt, cap, j, r0, lane, pv, hitlog, nlog, log_cap, flags);
        bT = rT;
        bgT = rgT;
        bA = rA;
        if ((t % kRescaleEvery) == kRescaleEvery - 1) {
            T mh = T(0), mp = T(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                mh = qmax(mh, qmax(Tp[r], qmax(bV1[r], bV2[r])));
                mp = qmax(mp, qmax(gTp[r], gbV[r]));
            }
            const int sh = -qexp(mh), sp = -qexp(mp);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bV1[r] = qldexp(bV1[r], sh); bV2[r] = qldexp(bV2[r], sh); Tp[r] = qldexp(Tp[r], sh);
                gbV[r] = qldexp(gbV[r], sp); gTp[r] = qldexp(gTp[r], sp);
            }
            oU1 = qldexp(oU1, sh); oU2 = qldexp(oU2, sh); bT = qldexp(bT, sh);
            ogU = qldexp(ogU, sp); bgT = qldexp(bgT, sp);
            FH -= sh;
            FP -= sp;
        }
    };
    // two steps per trip, the prefetch buffers swapping roles, so the loads
    // of one step are first waited for where the next step uses them
    int t = 0;
    for (; t + 1 < S; t += 2) {
        step(t, fa, ea, fb, eb);
        __builtin_amdgcn_sched_barrier(0);
        step(t + 1, fb, eb, fa, ea);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (t < S) step(t, fa, ea, fb, eb);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = lane * R + r;
        if (!trp && used && row < rows) {
            int c = cnt[r];
            if (c > cap) {
                atomicOr(flags, 2);
                c = cap;
            }
            rowcnt[r0 + row] = c;
        }
    }
    if (FIRST) a11 = rdlane(A[0], 0);
}

// ------------------------------------------------- end of one pair
// Row counts -> row pointers, the pair's block of the output pool, per-pair
// scalars, and the logged hits placed in row / column order.
__device__ void finish_pair(const PairArgs& a, int lane, int64_t p, int m, int n, int32_t* __restrict__ rp,
                            const int4* __restrict__ hitlog, int nlog, double zH, int ezH, double zP, int ezP,
                            double a11) {
    // ---- row counts -> row pointers (inclusive scan in place)
    int carry = 0;
    for (int base = 0; base < m; base += kWave) {
        const int idx = base + lane;
        int v = idx < m ? rp[1 + idx] : 0;
        v = wave_incl_scan(v, lane);
        if (idx < m) rp[1 + idx] = v + carry;
        carry += __shfl(v, kWave - 1, kWave);
    }
    if (lane == 0) rp[0] = 0;
    __threadfence_block();
    const int nnz = carry;
    // every lane takes part in the atomic (lane 0 adds the pair's entries),
    // so the wave-wide read of lane 0's result follows no branch on the lane
    const unsigned long long got = atomicAdd(a.pool_head, lane == 0 ? (unsigned long long)nnz : 0ull);
    const unsigned long long base =
        ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(got >> 32)) << 32) |
        (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(got & 0xffffffffull));
    if (lane == 0) {
        a.pair_nnz[p] = nnz;
        a.pair_base[p] = (int64_t)base;
        const double lzh = log((double)zH) + (double)ezH * 0.69314718055994530942;
        const double lzp = log((double)zP) + (double)ezP * 0.69314718055994530942;
        a.logz[2 * p] = lzh;
        a.logz[2 * p + 1] = lzp;
        a.dist[p] = 1.0 - a11 / (double)min(m, n);
    }
    // counts are written by the backward pass and bounded by cap, so a
    // negative total cannot occur on a complete pass; it is refused anyway,
    // since a wrapped total would pass the capacity test below
    if (nnz < 0 || (int64_t)base + nnz > a.pool_cap) {
        if (lane == 0) atomicOr(a.flags, 1);
        return;
    }
    // place the logged hits: the backward pass meets a row's columns in
    // decreasing order, so rank k from the row's end lands at
    // base + row_end - 1 - k (rows ascending, columns ascending)
    for (int e = lane; e < nlog; e += kWave) {
        const int4 h = hitlog[e];
        const int64_t pos = (int64_t)base + rp[h.x + 1] - 1 - h.y;
        a.pool_col[pos] = h.z;
        a.pool_val[pos] = __int_as_float(h.w);
    }
    __threadfence_block();
}

// ------------------------------------------------------------ one pair
// Output row counts of a transposed pair: the LDS column counts, cut to
// the row capacity (and reported past it), become the row counts the
// output's row pointers are scanned from.
__device__ __forceinline__ void zero_col_counts(int lane, int n, int* __restrict__ colcnt) {
    for (int jj = lane; jj < n; jj += kWave) colcnt[jj] = 0;
}
__device__ __forceinline__ void col_counts_to_rows(const PairArgs& a, int lane, int n, int cap,
                                                   const int* __restrict__ colcnt, int32_t* __restrict__ rowcnt) {
    for (int jj = lane; jj < n; jj += kWave) {
        int c = colcnt[jj];
        if (c > cap) {
            atomicOr(a.flags, 2);
            c = cap;
        }
        rowcnt[jj] = c;
    }
}
// entries an output row of the pair may hold: the class's staging capacity,
// or for a transposed pair min(its rows, floor(1 / thresh) + 1)
__device__ __forceinline__ int out_row_cap(const PairArgs& a, bool trp, int m) {
    return trp ? min(m, a.cap_thresh) : a.cap;
}

// Forward sweep over the bands top to bottom, backward sweep bottom to top,
// then the pair's output.  RB rows per lane, bands of kWave * RB rows.  A
// transposed pair (trp) is swept with the second sequence as x: the output
// rows are then the sweep's columns, counted in colcnt.
template <int RB, typename T, bool MULTI>
__device__ __forceinline__ void pair_bands(const PairArgs& a, int lane, char* slot,
                                           const typename Pair2<T>::type* tab, const Coef<T>& k, int64_t p, int m,
                                           int n, const uint8_t* x, const uint8_t* y, bool trp,
                                           int* __restrict__ colcnt) {
    using V2 = typename Pair2<T>::type;
    const int H = kWave * RB;
    const int nb = MULTI ? (m + H - 1) / H : 1;
    V2* spill = reinterpret_cast<V2*>(slot);
    int2* exps = reinterpret_cast<int2*>(slot + a.off_exps);
    FwdBnd<T>* fb = reinterpret_cast<FwdBnd<T>*>(slot + a.off_fb);
    BwdBnd<T>* bb = reinterpret_cast<BwdBnd<T>*>(slot + a.off_bb);
    int4* hitlog = reinterpret_cast<int4*>(slot + a.off_log);
    const int log_cap = (int)((a.slot_bytes - a.off_log) / (int64_t)sizeof(int4));
    int nlog = 0;

    T zH = T(1), zP = T(1);
    int ezH = 0, ezP = 0;
    const Col0* col0 = reinterpret_cast<const Col0*>(a.col0);
    for (int b = 0; b < nb; ++b) {
        const int r0 = b * H;
        const int rows = min(H, m - r0);
        const int L = (rows + RB - 1) / RB;
        V2* sp = spill + (int64_t)b * a.spill_band_stride;
        int2* ex = exps + (int64_t)b * a.exps_band_stride;
        const FwdBnd<T>* fi = fb + (int64_t)((b + 1) & 1) * a.bnd_stride;
        FwdBnd<T>* fo = fb + (int64_t)(b & 1) * a.bnd_stride;
        // the top band's position is fixed at compile time (its lane 0
        // starts from the begin state, the others from a boundary record:
        // different live values), the bottom band's is a runtime flag
        if (!MULTI)
            fwd_band<RB, T, 1, 1>(lane, x, y, n, r0, rows, L, tab, k, col0, sp, ex, fi, fo, zH, zP, ezH, ezP, true,
                                  true);
        else if (b == 0)
            fwd_band<RB, T, 1, kBandRuntime>(lane, x, y, n, r0, rows, L, tab, k, col0, sp, ex, fi, fo, zH, zP, ezH,
                                             ezP, true, nb == 1);
        else
            fwd_band<RB, T, 0, kBandRuntime>(lane, x, y, n, r0, rows, L, tab, k, col0, sp, ex, fi, fo, zH, zP, ezH,
                                             ezP, false, b == nb - 1);
        __threadfence_block();
    }
    const T invZH = T(a.consts->w_hmm) / zH;
    const T invZP = T(1.0 - a.consts->w_hmm) / zP;
    int32_t* rp = a.row_ptr + a.row_off[p];
    double a11 = 0.0;
    const int ocap = out_row_cap(a, trp, m);
    if (trp) zero_col_counts(lane, n, colcnt);
    for (int b = nb - 1; b >= 0; --b) {
        const int r0 = b * H;
        const int rows = min(H, m - r0);
        const int L = (rows + RB - 1) / RB;
        const V2* sp = spill + (int64_t)b * a.spill_band_stride;
        const int2* ex = exps + (int64_t)b * a.exps_band_stride;
        const BwdBnd<T>* bi = bb + (int64_t)((b + 1) & 1) * a.bnd_stride;
        BwdBnd<T>* bo = bb + (int64_t)(b & 1) * a.bnd_stride;
        // here the bottom band's position is the compile-time one (the
        // lane L-1 below it reads a boundary record or nothing)
        if (!MULTI)
            bwd_band<RB, T, 1, 1>(lane, x, y, n, r0, rows, L, tab, k, sp, ex, bi, bo, invZH, invZP, ezH, ezP,
                                  a.thresh, ocap, hitlog, nlog, rp + 1, a.flags, a11, true, true, trp, colcnt,
                                  log_cap);
        else if (b == nb - 1)
            bwd_band<RB, T, kBandRuntime, 1>(lane, x, y, n, r0, rows, L, tab, k, sp, ex, bi, bo, invZH, invZP, ezH,
                                             ezP, a.thresh, ocap, hitlog, nlog, rp + 1, a.flags, a11, b == 0, true,
                                             trp, colcnt, log_cap);
        else
            bwd_band<RB, T, kBandRuntime, 0>(lane, x, y, n, r0, rows, L, tab, k, sp, ex, bi, bo, invZH, invZP, ezH,
                                             ezP, a.thresh, ocap, hitlog, nlog, rp + 1, a.flags, a11, b == 0, false,
                                             trp, colcnt, log_cap);
        __threadfence_block();
    }
    if (trp) col_counts_to_rows(a, lane, n, ocap, colcnt, rp + 1);
    finish_pair(a, lane, p, trp ? n : m, trp ? m : n, rp, hitlog, nlog, (double)zH, ezH, (double)zP, ezP, a11);
}

// the pair's two sequences in the order it is swept: x (rows), y (columns)
struct PairSeqs {
    int xi, yi;
    bool trp;
};
__device__ __forceinline__ PairSeqs pair_seqs(const PairArgs& a, int64_t p) {
    const int pi = __builtin_amdgcn_readfirstlane(a.pair_i[p]);
    const int pj = __builtin_amdgcn_readfirstlane(a.pair_j[p]);
    const bool trp = a.tr && __builtin_amdgcn_readfirstlane((int)a.tr[p]) != 0;
    return PairSeqs{trp ? pj : pi, trp ? pi : pj, trp};
}

template <int R, typename T, bool MULTI>
__device__ __forceinline__ void process_pair(const PairArgs& a, int lane, char* slot,
                                             const typename Pair2<T>::type* tab, const Coef<T>& k, int64_t p,
                                             int* __restrict__ colcnt) {
    const PairSeqs ps = pair_seqs(a, p);
    const int m = __builtin_amdgcn_readfirstlane(a.lens[ps.xi]);
    const int n = __builtin_amdgcn_readfirstlane(a.lens[ps.yi]);
    const uint8_t* x = a.seqs + uniform64(a.seq_off[ps.xi]);
    const uint8_t* y = a.seqs + uniform64(a.seq_off[ps.yi]);
    pair_bands<R, T, MULTI>(a, lane, slot, tab, k, p, m, n, x, y, ps.trp, colcnt);
}

// One persistent launch per kernel class: waves pop pairs of their class
// from the cost-ordered queue segment (most expensive first).
template <int R, typename T, bool MULTI>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void k_pairs(PairArgs a) {
    using V2 = typename Pair2<T>::type;
    __shared__ V2 tab[kTabRows * kTabW];
    __shared__ int colcnt_s[kWavesPerBlock * kMaxSeqLen];  // output row counts of a transposed pair
    const V2* gtab = reinterpret_cast<const V2*>(a.tab);
    for (int t = threadIdx.x; t < kTabRows * kTabW; t += blockDim.x) tab[t] = gtab[t];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    // wave index is uniform: keep the slot pointer (and all pointers derived
    // from it) in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    char* slot = a.scratch + (int64_t)wid * a.slot_bytes;
    const DevConsts c = *a.consts;
    Coef<T> k;
    k.tau = (T)c.tau; k.eps1 = (T)c.eps1; k.eps2 = (T)c.eps2; k.c1 = (T)c.c1; k.c2 = (T)c.c2;
    k.u = (T)c.u; k.o = (T)c.o;
    // this class's queue segment: keys [cls*kCostBins, cls*kCostBins + kCostBins)
    const int k0 = a.cls * kCostBins, k1 = k0 + kCostBins - 1;
    const int seg_begin = __builtin_amdgcn_readfirstlane(a.bin_start[k1]);
    const int seg_end = __builtin_amdgcn_readfirstlane(a.bin_start[k0] + a.hist[k0]);
    int* head = a.queue_head + a.cls;
    for (;;) {
        // every lane takes part in the atomic (lane 0 adds one, the others
        // nothing), so no branch on the lane index comes before the wave-wide
        // read of its result that the compiler could route some lanes around;
        // wave-uniform from here on: scalar registers and scalar branches
        const int q = __builtin_amdgcn_readfirstlane(atomicAdd(head, lane == 0 ? 1 : 0)) + seg_begin;
        if (q >= seg_end) break;
        const int64_t p = __builtin_amdgcn_readfirstlane(a.queue[q]);
        process_pair<R, T, MULTI>(a, lane, slot, tab, k, p, colcnt_s + (threadIdx.x >> 6) * kMaxSeqLen);
    }
}

// Plain per-pair form: one launch of one wave per pair, no queue.  The host
// issues one launch per pair on a single stream, so every launch can use
// scratch slot 0 of its class.
template <int R, typename T, bool MULTI>
__global__ __launch_bounds__(kWave) void k_pair_one(PairArgs a, int64_t p) {
    using V2 = typename Pair2<T>::type;
    __shared__ V2 tab[kTabRows * kTabW];
    __shared__ int colcnt_s[kMaxSeqLen];
    const V2* gtab = reinterpret_cast<const V2*>(a.tab);
    for (int t = threadIdx.x; t < kTabRows * kTabW; t += blockDim.x) tab[t] = gtab[t];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const DevConsts c = *a.consts;
    Coef<T> k;
    k.tau = (T)c.tau; k.eps1 = (T)c.eps1; k.eps2 = (T)c.eps2; k.c1 = (T)c.c1; k.c2 = (T)c.c2;
    k.u = (T)c.u; k.o = (T)c.o;
    process_pair<R, T, MULTI>(a, lane, a.scratch, tab, k, p, colcnt_s);
}

// ======================================================= checkpointed form
// FP32 pair routine that keeps no per-cell value in memory.  The forward
// sweep saves its whole state (FwdSt) at the start of every block of
// kRescaleEvery steps, right after the block boundary's rescale, and writes
// nothing per cell; the backward sweep walks the blocks from the last one,
// restores a block's state, recomputes that block's forward match values
// into registers and consumes them in reverse step order.  The recomputed
// values are bit-identical to the first sweep's (same state, same
// arithmetic), so the posteriors are those of the spilling routine above;
// per cell the memory traffic drops from the 16-byte value pair written and
// read back to a (5R+13)-word state per lane and block.
//
// The backward sweep's rescale closes every block (instead of every eighth
// backward step), and its per-step work reads no memory.
// band position of a routine: 0 / 1 fixed at compile time (single-band
// kernels), 2 given at run time (the banded kernel keeps one instance of
// each routine instead of one per top / middle / bottom band)

template <int R> struct FwdSt {
    float W1[R], W2[R], D[R], gW[R], gD[R];
    float oM, oU1, oU2, ogM, ogU, aD, gaD, tv1, tv2, tgv;
    int EH, EP;
    FwdBnd<float> bq;
};
// 32-bit words of one lane's saved state
__host__ __device__ constexpr int ck_words(int R) { return 5 * R + 12; }
// The column sequence of the pair being processed sits in LDS (one region
// per wave) with kYPad zero bytes before and after it, so that every lane
// reads the residue of its own column, in or out of range, with one LDS byte
// load: no scalar load or lane-to-lane hand-over of residues in the step
// loops, and LDS waits there count LDS operations only.
constexpr int kYPad = kWave;
constexpr int kYStride = kMaxSeqLen + 2 * kYPad;

// state after column 0 of a band (before step 0)
template <int R, int FM, int LM>
__device__ __forceinline__ void ck_init(FwdSt<R>& f, int lane, bool used, int r0, int rows, int L,
                                        const Coef<float>& k, const Col0* __restrict__ col0,
                                        const FwdBnd<float>* __restrict__ fin, FwdBnd<float>* __restrict__ fout,
                                        bool rt_first, bool rt_last) {
    const bool FIRST = band_is(FM, rt_first), LAST = band_is(LM, rt_last);
    Col0 c0[R];
    int EH = INT_MIN, EP = INT_MIN;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = lane * R + r;
        if (used && row < rows) {
            c0[r] = col0[r0 + row];
        } else {
            c0[r].mH = 0.0;
            c0[r].mP = 0.0;
            c0[r].eH = 0;
            c0[r].eP = 0;
        }
        EH = max(EH, c0[r].mH != 0.0 ? c0[r].eH : INT_MIN);
        EP = max(EP, c0[r].mP != 0.0 ? c0[r].eP : INT_MIN);
    }
    if (EH == INT_MIN) EH = 0;
    if (EP == INT_MIN) EP = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        f.W1[r] = 0.f;
        f.W2[r] = 0.f;
        f.gW[r] = 0.f;
        f.D[r] = qldexp((float)c0[r].mH, c0[r].eH - EH);
        f.gD[r] = qldexp((float)c0[r].mP, c0[r].eP - EP);
    }
    f.EH = EH;
    f.EP = EP;
    f.oM = f.oU1 = f.oU2 = f.ogM = f.ogU = 0.f;
    f.aD = f.gaD = 0.f;
    f.tv1 = f.tv2 = f.tgv = 0.f;
    if (lane == 0) {
        if (FIRST) {
            f.aD = qldexp(k.tau, -EH);
            f.gaD = qldexp(1.f, -EP);
            f.tv1 = qldexp(1.f, -EH);
            f.tv2 = f.tv1;
            f.tgv = qldexp(1.f, -EP);
        } else {
            const FwdBnd<float> b = fin[0];
            f.aD = qldexp(b.D, b.EH - EH);
            f.gaD = qldexp(b.gD, b.EP - EP);
        }
    }
    if (!LAST && lane == L - 1) {
        FwdBnd<float> b;
        b.M = 0.f; b.U1 = 0.f; b.U2 = 0.f; b.D = f.D[R - 1];
        b.gM = 0.f; b.gU = 0.f; b.gD = f.gD[R - 1];
        b.EH = EH; b.EP = EP;
        fout[0] = b;
    }
    if (!FIRST && lane == 0) f.bq = fin[1];
}

// one forward step: the match values of the lane's rows at its column go to
// sm; WB: also write the band's boundary record (first sweep only)
// (ycn: the residue of this step's column, read one step ahead; the read
// for the next step is issued here)
template <int R, int FM, int LM, bool WB>
__device__ __forceinline__ void ck_fstep(FwdSt<R>& f, float2 (&sm)[R], const int s, const int lane, const bool used,
                                         const int n, const int L, const int (&xo)[R], const uint8_t* ys,
                                         int& ycn, const float2* tab, const Coef<float>& k,
                                         const FwdBnd<float>* __restrict__ fin, FwdBnd<float>* __restrict__ fout,
                                         bool rt_first, bool rt_last) {
    const bool FIRST = band_is(FM, rt_first), LAST = band_is(LM, rt_last);
    const int j = s - lane + 1;
    const bool active = used && j >= 1 && j <= n;
    const int yc = ycn;
    ycn = ys[j];
    float rM = dpp<kDppWaveShr1>(f.oM), rU1 = dpp<kDppWaveShr1>(f.oU1), rU2 = dpp<kDppWaveShr1>(f.oU2);
    float rD = dpp<kDppWaveShr1>(f.D[R - 1]), rgM = dpp<kDppWaveShr1>(f.ogM), rgU = dpp<kDppWaveShr1>(f.ogU);
    float rgD = dpp<kDppWaveShr1>(f.gD[R - 1]);
    int rEH = dpp_i<kDppWaveShr1>(f.EH), rEP = dpp_i<kDppWaveShr1>(f.EP);
    if (lane == 0) {
        if (FIRST) {
            rM = 0.f; rU1 = 0.f; rU2 = 0.f;
            rD = k.c1 * f.tv1 + k.c2 * f.tv2;
            rgM = 0.f; rgU = 0.f;
            rgD = k.o * f.tgv;
            rEH = f.EH; rEP = f.EP;
            f.tv1 *= k.eps1; f.tv2 *= k.eps2; f.tgv *= k.u;
        } else {
            rM = f.bq.M; rU1 = f.bq.U1; rU2 = f.bq.U2; rD = f.bq.D;
            rgM = f.bq.gM; rgU = f.bq.gU; rgD = f.bq.gD;
            rEH = f.bq.EH; rEP = f.bq.EP;
            f.bq = fin[s + 2 <= n ? s + 2 : n];
        }
    }
    {
        const int dH = rEH - f.EH, dP = rEP - f.EP;
        rM = qldexp(rM, dH); rU1 = qldexp(rU1, dH); rU2 = qldexp(rU2, dH); rD = qldexp(rD, dH);
        rgM = qldexp(rgM, dP); rgU = qldexp(rgU, dP); rgD = qldexp(rgD, dP);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float2 e = tab[xo[r] + yc];
        sm[r].x = e.x * (r == 0 ? f.aD : f.D[r - 1]);
        sm[r].y = e.y * (r == 0 ? f.gaD : f.gD[r - 1]);
    }
    f.oM = sm[R - 1].x;
    f.ogM = sm[R - 1].y;
    if (active) {
        float upM = rM, upU1 = rU1, upU2 = rU2;
        float gupM = rgM, gupU = rgU;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float nM = sm[r].x, ngM = sm[r].y;
            const float nU1 = fmaf(k.eps1, upU1, upM);
            const float nU2 = fmaf(k.eps2, upU2, upM);
            f.D[r] = fmaf(k.c2, nU2 + f.W2[r], fmaf(k.c1, nU1 + f.W1[r], k.tau * nM));
            const float ngU = fmaf(k.u, gupU, gupM);
            f.gD[r] = fmaf(k.o, ngU + f.gW[r], ngM);
            f.W1[r] = fmaf(k.eps1, f.W1[r], nM);
            f.W2[r] = fmaf(k.eps2, f.W2[r], nM);
            f.gW[r] = fmaf(k.u, f.gW[r], ngM);
            upM = nM; upU1 = nU1; upU2 = nU2;
            gupM = ngM; gupU = ngU;
        }
        f.oU1 = upU1; f.oU2 = upU2;
        f.ogU = gupU;
        if (WB && !LAST && lane == L - 1) {
            FwdBnd<float> b;
            b.M = f.oM; b.U1 = f.oU1; b.U2 = f.oU2; b.D = f.D[R - 1];
            b.gM = f.ogM; b.gU = f.ogU; b.gD = f.gD[R - 1];
            b.EH = f.EH; b.EP = f.EP;
            fout[j] = b;
        }
    }
    f.aD = rD;
    f.gaD = rgD;
}

// power-of-two rescale at a block boundary (as the spilling sweep's)
template <int R>
__device__ __forceinline__ void ck_frescale(FwdSt<R>& f) {
    float mh = 0.f, mp = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        mh = fmaxf(mh, f.D[r]);
        mp = fmaxf(mp, f.gD[r]);
    }
    const int sh = -qexp(mh), sp = -qexp(mp);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        f.W1[r] = qldexp(f.W1[r], sh); f.W2[r] = qldexp(f.W2[r], sh); f.D[r] = qldexp(f.D[r], sh);
        f.gW[r] = qldexp(f.gW[r], sp); f.gD[r] = qldexp(f.gD[r], sp);
    }
    f.oM = qldexp(f.oM, sh); f.oU1 = qldexp(f.oU1, sh); f.oU2 = qldexp(f.oU2, sh);
    f.aD = qldexp(f.aD, sh); f.tv1 = qldexp(f.tv1, sh); f.tv2 = qldexp(f.tv2, sh);
    f.ogM = qldexp(f.ogM, sp); f.ogU = qldexp(f.ogU, sp);
    f.gaD = qldexp(f.gaD, sp); f.tgv = qldexp(f.tgv, sp);
    f.EH -= sh;
    f.EP -= sp;
}

// saved state of one block: word w of lane l at ck[w * kWave + l]
__device__ __forceinline__ void ck_put(float* ck, int w, int lane, float v) {
    __builtin_nontemporal_store(v, ck + w * kWave + lane);
}
__device__ __forceinline__ float ck_get(const float* ck, int w, int lane) {
    return __builtin_nontemporal_load(ck + w * kWave + lane);
}
template <int R, int FM>
__device__ __forceinline__ void ck_save(const FwdSt<R>& f, float* ck, int lane, bool rt_first) {
    const bool FIRST = band_is(FM, rt_first);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ck_put(ck, r, lane, f.W1[r]);
        ck_put(ck, R + r, lane, f.W2[r]);
        ck_put(ck, 2 * R + r, lane, f.D[r]);
        ck_put(ck, 3 * R + r, lane, f.gW[r]);
        ck_put(ck, 4 * R + r, lane, f.gD[r]);
    }
    const int b = 5 * R;
    ck_put(ck, b + 0, lane, f.oM);
    ck_put(ck, b + 1, lane, f.oU1);
    ck_put(ck, b + 2, lane, f.oU2);
    ck_put(ck, b + 3, lane, f.ogM);
    ck_put(ck, b + 4, lane, f.ogU);
    ck_put(ck, b + 5, lane, f.aD);
    ck_put(ck, b + 6, lane, f.gaD);
    if (FIRST) {
        ck_put(ck, b + 7, lane, f.tv1);
        ck_put(ck, b + 8, lane, f.tv2);
        ck_put(ck, b + 9, lane, f.tgv);
    }
    ck_put(ck, b + 10, lane, __int_as_float(f.EH));
    ck_put(ck, b + 11, lane, __int_as_float(f.EP));
}
template <int R, int FM>
__device__ __forceinline__ void ck_load(FwdSt<R>& f, const float* ck, int lane, bool rt_first) {
    const bool FIRST = band_is(FM, rt_first);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        f.W1[r] = ck_get(ck, r, lane);
        f.W2[r] = ck_get(ck, R + r, lane);
        f.D[r] = ck_get(ck, 2 * R + r, lane);
        f.gW[r] = ck_get(ck, 3 * R + r, lane);
        f.gD[r] = ck_get(ck, 4 * R + r, lane);
    }
    const int b = 5 * R;
    f.oM = ck_get(ck, b + 0, lane);
    f.oU1 = ck_get(ck, b + 1, lane);
    f.oU2 = ck_get(ck, b + 2, lane);
    f.ogM = ck_get(ck, b + 3, lane);
    f.ogU = ck_get(ck, b + 4, lane);
    f.aD = ck_get(ck, b + 5, lane);
    f.gaD = ck_get(ck, b + 6, lane);
    if (FIRST) {
        f.tv1 = ck_get(ck, b + 7, lane);
        f.tv2 = ck_get(ck, b + 8, lane);
        f.tgv = ck_get(ck, b + 9, lane);
    } else {
        f.tv1 = f.tv2 = f.tgv = 0.f;
    }
    f.EH = __float_as_int(ck_get(ck, b + 10, lane));
    f.EP = __float_as_int(ck_get(ck, b + 11, lane));
}

// first sweep of one band: the state at every block start goes to ck, the
// boundary records of a band above the last to fout; Z from the last band
template <int R, int FM, int LM>
__device__ void ck_fwd_band(int lane, const uint8_t* __restrict__ x, const uint8_t* ys, int n, int r0,
                            int rows, int L, const float2* tab, const Coef<float>& k,
                            const Col0* __restrict__ col0, float* __restrict__ ck,
                            const FwdBnd<float>* __restrict__ fin, FwdBnd<float>* __restrict__ fout, float& zH,
                            float& zP, int& ezH, int& ezP, bool rt_first, bool rt_last) {
    const bool LAST = band_is(LM, rt_last);
    const bool used = lane < L;
    int xo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = lane * R + r;
        xo[r] = (used && row < rows ? (int)x[r0 + row] : kPadCode) * kTabW;
    }
    FwdSt<R> f;
    ck_init<R, FM, LM>(f, lane, used, r0, rows, L, k, col0, fin, fout, rt_first, rt_last);
    const int S = n + L - 1;
    float2 sm[R];
    int ycn = ys[-lane];
    for (int s0 = 0, blk = 0; s0 < S; s0 += kRescaleEvery, ++blk) {
        ck_save<R, FM>(f, ck + (int64_t)blk * ck_words(R) * kWave, lane, rt_first);
        if (s0 + kRescaleEvery <= S) {
#pragma unroll
            for (int q = 0; q < kRescaleEvery; ++q)
                ck_fstep<R, FM, LM, true>(f, sm, s0 + q, lane, used, n, L, xo, ys, ycn, tab, k, fin, fout, rt_first,
                                          rt_last);
            ck_frescale<R>(f);
        } else {
            for (int s = s0; s < S; ++s)
                ck_fstep<R, FM, LM, true>(f, sm, s, lane, used, n, L, xo, ys, ycn, tab, k, fin, fout, rt_first, rt_last);
        }
    }
    if (LAST) {
        const int rm = (rows - 1) - (L - 1) * R;
        float zd = 0.f, zg = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r == rm) { zd = f.D[r]; zg = f.gD[r]; }
        zH = rdlane(zd, L - 1);
        zP = rdlane(zg, L - 1);
        ezH = rdlane(f.EH, L - 1);
        ezP = rdlane(f.EP, L - 1);
    }
}

// backward sweep of one band with the forward values recomputed per block
// (a whole block of values held in registers)
template <int R, int FM, int LM>
__device__ void ck_bwd_band(int lane, const uint8_t* __restrict__ x, const uint8_t* ys, int n, int r0,
                            int rows, int L, const float2* tab, const Coef<float>& k,
                            const float* __restrict__ ck, const FwdBnd<float>* __restrict__ fin,
                            const BwdBnd<float>* __restrict__ bin, BwdBnd<float>* __restrict__ bout, float invZH,
                            float invZP, int ezH, int ezP, float thresh, int cap, int4* __restrict__ hitlog,
                            int& nlog, int32_t* __restrict__ rowcnt, int* __restrict__ flags, double& a11,
                            bool rt_first, bool rt_last, bool trp, int* __restrict__ colcnt, int log_cap) {
    const bool FIRST = band_is(FM, rt_first), LAST = band_is(LM, rt_last);
    const bool used = lane < L;
    int xo[R];
    bool inrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = lane * R + r;
        inrow[r] = used && row < rows;
        xo[r] = (inrow[r] ? (int)x[r0 + row] : kPadCode) * kTabW;
    }
    float bV1[R], bV2[R], Tp[R], gbV[R], gTp[R];
    double A[R];
    int cnt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bV1[r] = 0.f; bV2[r] = 0.f; Tp[r] = 0.f; gbV[r] = 0.f; gTp[r] = 0.f;
        A[r] = 0.0;
        cnt[r] = 0;
    }
    int FH = 0, FP = 0;
    float bT = 0.f, bgT = 0.f;
    double bA = 0.0;
    if (LAST && lane == L - 1) {
        const int rm = (rows - 1) - (L - 1) * R;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r == rm + 1) { Tp[r] = invZH; gTp[r] = invZP; }
        if (rm + 1 == R) { bT = invZH; bgT = invZP; }
    }
    float oU1 = 0.f, oU2 = 0.f, ogU = 0.f;
    const int S = n + L - 1;
    const int lead = L - 1 - lane;
    BwdBnd<float> bq;
    if (!LAST && lane == L - 1) bq = bin[n];

    // backward step t with the forward values fc of forward step S-1-t,
    // whose exponents are ec.  Every lane computes every step: a lane that
    // has not reached its first column holds zeros and receives zeros, and a
    // lane past its last column computes values no active lane reads, so
    // only the hit counts, the logged hits and the band boundary record are
    // kept to the lane's own columns.
    int ybn = ys[n + lead - 1];  // residue of the next backward step's column
    auto bstep = [&](const int t, const float2 (&fc)[R], const int2 ec) {
        const int j = n - t + lead;
        const bool active = used && j >= 1 && j <= n;
        const int yc = ybn;
        ybn = ys[j - 2];
        float rU1 = dpp<kDppWaveShl1>(oU1), rU2 = dpp<kDppWaveShl1>(oU2), rT = dpp<kDppWaveShl1>(Tp[0]);
        float rgU = dpp<kDppWaveShl1>(ogU), rgT = dpp<kDppWaveShl1>(gTp[0]);
        double rA = dpp<kDppWaveShl1>(A[0]);
        int rFH = dpp_i<kDppWaveShl1>(FH), rFP = dpp_i<kDppWaveShl1>(FP);
        if (!LAST) {
            // lane L-1 of a band above the last takes the lower band's record;
            // in the last band, lane L-1 reads an unused lane (zeros), which
            // is what lies below the last row
            const bool edge = lane == L - 1;
            rU1 = edge ? bq.U1 : rU1;
            rU2 = edge ? bq.U2 : rU2;
            rT = edge ? bq.Tt : rT;
            rgU = edge ? bq.gU : rgU;
            rgT = edge ? bq.gT : rgT;
            rA = edge ? bq.A : rA;
            rFH = edge ? bq.FH : rFH;
            rFP = edge ? bq.FP : rFP;
            if (edge) bq = bin[j - 1 >= 1 ? j - 1 : 1];
        }
        {
            const bool adopt = j >= n && !(LAST && lane == L - 1);
            const int nFH = adopt ? rFH : FH, nFP = adopt ? rFP : FP;
            bT = qldexp(bT, FH - nFH);
            bgT = qldexp(bgT, FP - nFP);
            FH = nFH;
            FP = nFP;
            const int dH = rFH - FH, dP = rFP - FP;
            rU1 = qldexp(rU1, dH); rU2 = qldexp(rU2, dH); rT = qldexp(rT, dH);
            rgU = qldexp(rgU, dP); rgT = qldexp(rgT, dP);
        }
        int hbits = 0;  // rows of this step with a hit
        float pv[R];
        {
            float dU1 = rU1, dU2 = rU2, dgU = rgU;
            double dA = rA;
            float dgT = bT, dggT = bgT;
            double dgA = bA;
            const int kH = ec.x + FH - ezH, kP = ec.y + FP - ezP;
#pragma unroll
            for (int r = R - 1; r >= 0; --r) {
                const float2 e = tab[xo[r] + yc];
                const float t1 = dgT, tg = dggT;
                const float nU1 = fmaf(k.eps1, dU1, t1);
                const float nU2 = fmaf(k.eps2, dU2, t1);
                const float nV1 = fmaf(k.eps1, bV1[r], t1);
                const float nV2 = fmaf(k.eps2, bV2[r], t1);
                const float bM = fmaf(k.c2, dU2 + bV2[r], fmaf(k.c1, dU1 + bV1[r], k.tau * t1));
                const float nT = e.x * bM;
                const float ngU = fmaf(k.u, dgU, tg);
                const float ngV = fmaf(k.u, gbV[r], tg);
                const float gbM = fmaf(k.o, dgU + gbV[r], tg);
                const float ngT = e.y * gbM;
                const float pH = qldexp(fc[r].x * bM, kH);
                const float pP = qldexp(fc[r].y * gbM, kP);
                const float P = pH + pP;
                const double nA = fmax(dgA + (double)P, fmax(dA, A[r]));
                const bool hit = active && inrow[r] && P >= thresh;
                pv[r] = P;
                cnt[r] += hit ? 1 : 0;
                hbits |= hit ? (1 << r) : 0;
                dgT = Tp[r]; dggT = gTp[r]; dgA = A[r];
                Tp[r] = nT; gTp[r] = ngT; A[r] = nA;
                bV1[r] = nV1; bV2[r] = nV2; gbV[r] = ngV;
                dU1 = nU1; dU2 = nU2; dgU = ngU; dA = nA;
            }
            oU1 = dU1; oU2 = dU2; ogU = dgU;
            if (!FIRST && lane == 0 && active) {
                BwdBnd<float> b;
                b.U1 = oU1; b.U2 = oU2; b.Tt = Tp[0]; b.gU = ogU; b.gT = gTp[0]; b.A = A[0];
                b.FH = FH; b.FP = FP;
                bout[j] = b;
            }
        }
        log_hits<R>(hbits, trp, colcnt, cnt, cap, j, r0, lane, pv, hitlog, nlog, log_cap, flags);
        bT = rT;
        bgT = rgT;
        bA = rA;
    };
    auto brescale = [&]() {
        float mh = 0.f, mp = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            mh = fmaxf(mh, fmaxf(Tp[r], fmaxf(bV1[r], bV2[r])));
            mp = fmaxf(mp, fmaxf(gTp[r], gbV[r]));
        }
        const int sh = -qexp(mh), sp = -qexp(mp);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bV1[r] = qldexp(bV1[r], sh); bV2[r] = qldexp(bV2[r], sh); Tp[r] = qldexp(Tp[r], sh);
            gbV[r] = qldexp(gbV[r], sp); gTp[r] = qldexp(gTp[r], sp);
        }
        oU1 = qldexp(oU1, sh); oU2 = qldexp(oU2, sh); bT = qldexp(bT, sh);
        ogU = qldexp(ogU, sp); bgT = qldexp(bgT, sp);
        FH -= sh;
        FP -= sp;
    };

    // one block of kRescaleEvery forward steps, consumed backwards; FULL:
    // the block has all its steps (no per-step guard, so values stay in
    // place between steps); the one partial block of a band, the last, is
    // handled by the guarded instance
    auto block = [&](const int blk, auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        const int s0 = blk * kRescaleEvery;
        const int ns = FULL ? kRescaleEvery : min(kRescaleEvery, S - s0);
        FwdSt<R> f;
        int ycn = ys[s0 - lane];
        ck_load<R, FM>(f, ck + (int64_t)blk * ck_words(R) * kWave, lane, rt_first);
        if (!FIRST && lane == 0) f.bq = fin[min(s0 + 1, n)];
        const int2 ec = make_int2(f.EH, f.EP);
        float2 buf[kRescaleEvery][R];
#pragma unroll
        for (int q = 0; q < kRescaleEvery; ++q)
            if (FULL || q < ns)
                ck_fstep<R, FM, LM, false>(f, buf[q], s0 + q, lane, used, n, L, xo, ys, ycn, tab, k, fin,
                                           nullptr, rt_first, rt_last);
#pragma unroll
        for (int q = kRescaleEvery - 1; q >= 0; --q)
            if (FULL || q < ns) bstep(S - 1 - (s0 + q), buf[q], ec);
        brescale();
    };
    int blk = (S + kRescaleEvery - 1) / kRescaleEvery - 1;
    if (S % kRescaleEvery != 0) block(blk--, std::false_type{});
    for (; blk >= 0; --blk) block(blk, std::true_type{});
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = lane * R + r;
        if (!trp && inrow[r]) {
            int c = cnt[r];
            if (c > cap) {
                atomicOr(flags, 2);
                c = cap;
            }
            rowcnt[r0 + row] = c;
        }
    }
    if (FIRST) a11 = rdlane(A[0], 0);
}

template <int R, bool MULTI>
__device__ __forceinline__ void process_pair_ck(const PairArgs& a, int lane, char* slot, const float2* tab, uint8_t* yreg,
                                const Coef<float>& k, int64_t p, int* __restrict__ colcnt) {
    const PairSeqs ps = pair_seqs(a, p);
    const bool trp = ps.trp;
    const int m = __builtin_amdgcn_readfirstlane(a.lens[ps.xi]);
    const int n = __builtin_amdgcn_readfirstlane(a.lens[ps.yi]);
    const uint8_t* x = a.seqs + uniform64(a.seq_off[ps.xi]);
    const uint8_t* y = a.seqs + uniform64(a.seq_off[ps.yi]);
    const int H = kWave * R;
    const int nb = MULTI ? (m + H - 1) / H : 1;
    // the column sequence into this wave's LDS region, zeros around it (the
    // wave's reads of the previous pair come before these writes in its
    // instruction stream)
    for (int i = lane; i < n + 2 * kYPad; i += kWave) {
        const int idx = i - kYPad;
        yreg[i] = idx >= 0 && idx < n ? y[idx] : (uint8_t)0;
    }
    const uint8_t* ys = yreg + kYPad;
    float* ck = reinterpret_cast<float*>(slot);
    FwdBnd<float>* fb = reinterpret_cast<FwdBnd<float>*>(slot + a.off_fb);
    BwdBnd<float>* bb = reinterpret_cast<BwdBnd<float>*>(slot + a.off_bb);
    int4* hitlog = reinterpret_cast<int4*>(slot + a.off_log);
    const int log_cap = (int)((a.slot_bytes - a.off_log) / (int64_t)sizeof(int4));
    int nlog = 0;
    float zH = 1.f, zP = 1.f;
    int ezH = 0, ezP = 0;
    const Col0* col0 = reinterpret_cast<const Col0*>(a.col0);
    // every band keeps its forward boundary records: the band below reads
    // them again when it recomputes its blocks in the backward sweep
    for (int b = 0; b < nb; ++b) {
        const int r0 = b * H;
        const int rows = min(H, m - r0);
        const int L = (rows + R - 1) / R;
        float* c = ck + (int64_t)b * a.spill_band_stride;
        const FwdBnd<float>* fi = fb + (int64_t)(b > 0 ? b - 1 : 0) * a.bnd_stride;
        FwdBnd<float>* fo = fb + (int64_t)b * a.bnd_stride;
        if (!MULTI)
            ck_fwd_band<R, 1, 1>(lane, x, ys, n, r0, rows, L, tab, k, col0, c, fi, fo, zH, zP, ezH, ezP, true, true);
        else
            ck_fwd_band<R, kBandRuntime, kBandRuntime>(lane, x, ys, n, r0, rows, L, tab, k, col0, c, fi, fo, zH, zP,
                                                       ezH, ezP, b == 0, b == nb - 1);
        __threadfence_block();
    }
    const float invZH = (float)a.consts->w_hmm / zH;
    const float invZP = (float)(1.0 - a.consts->w_hmm) / zP;
    int32_t* rp = a.row_ptr + a.row_off[p];
    double a11 = 0.0;
    const int ocap = out_row_cap(a, trp, m);
    if (trp) zero_col_counts(lane, n, colcnt);
    for (int b = nb - 1; b >= 0; --b) {
        const int r0 = b * H;
        const int rows = min(H, m - r0);
        const int L = (rows + R - 1) / R;
        const float* c = ck + (int64_t)b * a.spill_band_stride;
        const FwdBnd<float>* fi = fb + (int64_t)(b > 0 ? b - 1 : 0) * a.bnd_stride;
        const BwdBnd<float>* bi = bb + (int64_t)((b + 1) & 1) * a.bnd_stride;
        BwdBnd<float>* bo = bb + (int64_t)(b & 1) * a.bnd_stride;
        if (!MULTI)
            ck_bwd_band<R, 1, 1>(lane, x, ys, n, r0, rows, L, tab, k, c, fi, bi, bo, invZH, invZP, ezH, ezP, a.thresh,
                                 ocap, hitlog, nlog, rp + 1, a.flags, a11, true, true, trp, colcnt, log_cap);
        else
            ck_bwd_band<R, kBandRuntime, kBandRuntime>(lane, x, ys, n, r0, rows, L, tab, k, c, fi, bi, bo, invZH,
                                                       invZP, ezH, ezP, a.thresh, ocap, hitlog, nlog, rp + 1,
                                                       a.flags, a11, b == 0, b == nb - 1, trp, colcnt, log_cap);
        __threadfence_block();
    }
    if (trp) col_counts_to_rows(a, lane, n, ocap, colcnt, rp + 1);
    finish_pair(a, lane, p, trp ? n : m, trp ? m : n, rp, hitlog, nlog, (double)zH, ezH, (double)zP, ezP, a11);
}

template <int R, bool MULTI>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void k_pairs_ck(PairArgs a) {
    __shared__ float2 tab[kTabRows * kTabW];
    __shared__ uint8_t ysh[kWavesPerBlock * kYStride];
    __shared__ int colcnt_s[kWavesPerBlock * kMaxSeqLen];  // output row counts of a transposed pair
    const float2* gtab = reinterpret_cast<const float2*>(a.tab);
    for (int t = threadIdx.x; t < kTabRows * kTabW; t += blockDim.x) tab[t] = gtab[t];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    char* slot = a.scratch + (int64_t)wid * a.slot_bytes;
    const DevConsts c = *a.consts;
    Coef<float> k;
    k.tau = (float)c.tau; k.eps1 = (float)c.eps1; k.eps2 = (float)c.eps2; k.c1 = (float)c.c1; k.c2 = (float)c.c2;
    k.u = (float)c.u; k.o = (float)c.o;
    const int k0 = a.cls * kCostBins, k1 = k0 + kCostBins - 1;
    const int seg_begin = __builtin_amdgcn_readfirstlane(a.bin_start[k1]);
    const int seg_end = __builtin_amdgcn_readfirstlane(a.bin_start[k0] + a.hist[k0]);
    int* head = a.queue_head + a.cls;
    for (;;) {
        // the pop as in k_pairs
        const int q = __builtin_amdgcn_readfirstlane(atomicAdd(head, lane == 0 ? 1 : 0)) + seg_begin;
        if (q >= seg_end) break;
        const int64_t p = __builtin_amdgcn_readfirstlane(a.queue[q]);
        process_pair_ck<R, MULTI>(a, lane, slot, tab, ysh + (threadIdx.x >> 6) * kYStride, k, p,
                                  colcnt_s + (threadIdx.x >> 6) * kMaxSeqLen);
    }
}

template <int R, bool MULTI>
__global__ __launch_bounds__(kWave) void k_pair_one_ck(PairArgs a, int64_t p) {
    __shared__ float2 tab[kTabRows * kTabW];
    __shared__ uint8_t ysh[kYStride];
    __shared__ int colcnt_s[kMaxSeqLen];
    const float2* gtab = reinterpret_cast<const float2*>(a.tab);
    for (int t = threadIdx.x; t < kTabRows * kTabW; t += blockDim.x) tab[t] = gtab[t];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const DevConsts c = *a.consts;
    Coef<float> k;
    k.tau = (float)c.tau; k.eps1 = (float)c.eps1; k.eps2 = (float)c.eps2; k.c1 = (float)c.c1; k.c2 = (float)c.c2;
    k.u = (float)c.u; k.o = (float)c.o;
    process_pair_ck<R, MULTI>(a, lane, a.scratch, tab, ysh, k, p, colcnt_s);
}

// ------------------------------------------------------ tables (a2 step)
// Builds the (e_hmm, w_pf) table and the scaled constants from the raw
// parameters in FP64, rounding once to the kernel precision.
// D(i,0) = sum_k c_k eps_k^(i-1) and o u^(i-1), as mantissa/exponent pairs:
// log2 in FP64, exact power-of-two exponent split, mantissa rounded once
__device__ void col0_entry(const DevParams* p, int i0, Col0* out) {
    const int G = p->n_gap_classes;
    const double d1 = p->gap_open[0], e1 = p->gap_extend[0];
    const double d2 = G > 1 ? p->gap_open[1] : 0.0, e2 = G > 1 ? p->gap_extend[1] : 0.0;
    const double c1 = d1 * (1.0 - e1), c2 = d2 * (1.0 - e2);
    auto term = [&](double c, double e) -> double {  // log2(c e^i0), -inf if zero
        if (c <= 0.0) return -(double)INFINITY;
        if (i0 == 0) return log2(c);
        if (e <= 0.0) return -(double)INFINITY;
        return log2(c) + (double)i0 * log2(e);
    };
    const double a1 = term(c1, e1), a2 = term(c2, e2);
    const double am = fmax(a1, a2);
    Col0 r;
    if (am == -INFINITY) {
        r.mH = 0.0;
        r.eH = 0;
    } else {
        const int E = (int)floor(am);
        const double v = (a1 == -INFINITY ? 0.0 : exp2(a1 - E)) + (a2 == -INFINITY ? 0.0 : exp2(a2 - E));
        r.mH = v;
        r.eH = E;
    }
    const double o = exp(p->pf_gap_open / p->temperature), u = exp(p->pf_gap_extend / p->temperature);
    const double ap = log2(o) + (i0 == 0 ? 0.0 : (double)i0 * log2(u));
    const int EPp = (int)floor(ap);
    r.mP = exp2(ap - EPp);
    r.eP = EPp;
    *out = r;
}

template <typename T>
__global__ void k_tables(const DevParams* __restrict__ p, typename Pair2<T>::type* __restrict__ tab,
                         DevConsts* __restrict__ c, Col0* __restrict__ col0, int rows) {
    for (int i = (blockIdx.x - 1) * blockDim.x + threadIdx.x; blockIdx.x > 0 && i < rows;
         i += (gridDim.x - 1) * blockDim.x)
        col0_entry(p, i, &col0[i]);
    if (blockIdx.x > 0) return;
    using V2 = typename Pair2<T>::type;
    const int t = threadIdx.x;
    __shared__ double qx[20], qy[20];
    if (t < 20) {
        double sx = 0.0, sy = 0.0;
        for (int b = 0; b < 20; ++b) {
            sx += p->joint[t * 20 + b];
            sy += p->joint[b * 20 + t];
        }
        qx[t] = sx;
        qy[t] = sy;
    }
    __syncthreads();
    for (int idx = t; idx < kTabRows * kTabW; idx += blockDim.x) {
        const int a = idx / kTabW, b = idx % kTabW;
        V2 v;
        v.x = T(0);
        v.y = T(0);
        if (a < p->alphabet && b < p->alphabet) {  // other codes never occur (zero weight)
            v.x = (T)(p->joint[a * 20 + b] / (qx[a] * qy[b]));
            v.y = (T)exp(p->score[a * 20 + b] / p->temperature);
        }
        tab[idx] = v;
    }
    if (t == 0) {
        const int G = p->n_gap_classes;
        const double d1 = p->gap_open[0], e1 = p->gap_extend[0];
        const double d2 = G > 1 ? p->gap_open[1] : 0.0, e2 = G > 1 ? p->gap_extend[1] : 0.0;
        DevConsts k;
        k.tau = 1.0 - 2.0 * (d1 + d2);
        k.eps1 = e1;
        k.eps2 = e2;
        k.c1 = d1 * (1.0 - e1);
        k.c2 = d2 * (1.0 - e2);
        k.u = exp(p->pf_gap_extend / p->temperature);
        k.o = exp(p->pf_gap_open / p->temperature);
        k.w_hmm = p->w_hmm;
        *c = k;
    }
}

// -------------------------------------------------- schedule (a1 step)
__global__ void k_reset(int* ints, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ints[i] = 0;
}

__device__ __forceinline__ int64_t pair_start(int64_t i, int64_t n) { return i * n - i * (i + 1) / 2; }


// 4-byte aligned, zero padded copy of every sequence; codes outside the
// alphabet are reported through bit 4 of *flags (and copied as the padding
// code)
__global__ void k_stage_seqs(int32_t n, int32_t alphabet, const uint8_t* __restrict__ seqs, const int64_t* __restrict__ seq_off,
                             const int32_t* __restrict__ lens, const int64_t* __restrict__ seqa_off,
                             uint8_t* __restrict__ seqa, int* __restrict__ flags) {
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t src = seq_off[i], dst = seqa_off[i];
        const int len = lens[i], padded = (int)(seqa_off[i + 1] - dst);
        bool bad = false;
        for (int c = threadIdx.x; c < padded; c += blockDim.x) {
            const uint8_t v = c < len ? seqs[src + c] : (uint8_t)0;
            bad |= v >= alphabet;
            seqa[dst + c] = v >= alphabet ? (uint8_t)kPadCode : v;  // keeps table reads in range
        }
        if (bad) atomicOr(flags, 4);
    }
}

__global__ void k_setup(int32_t n, const int32_t* __restrict__ lens, const int32_t* __restrict__ list_i,
                        const int32_t* __restrict__ list_j, const uint8_t* __restrict__ tr, int64_t P,
                        int32_t* __restrict__ pi,
                        int32_t* __restrict__ pj, int64_t* __restrict__ rows1, int32_t* __restrict__ key,
                        int* __restrict__ hist, int64_t* __restrict__ pair_nnz, ClassMap map) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        rows1[P] = 0;
        pair_nnz[P] = 0;
    }
    // lanes past the pair list take part in the wave-wide count only
    int kk = 0;
    if (p < P) {
        int64_t i, j;
        if (list_i) {
            i = list_i[p];
            j = list_j[p];
        } else {
            const double nn = (double)n;
            const double disc = (2.0 * nn - 1.0) * (2.0 * nn - 1.0) - 8.0 * (double)p;
            i = (int64_t)floor((2.0 * nn - 1.0 - sqrt(disc > 0 ? disc : 0.0)) / 2.0);
            if (i < 0) i = 0;
            while (i > 0 && pair_start(i, n) > p) --i;
            while (i + 1 < n && pair_start(i + 1, n) <= p) ++i;
            j = p - pair_start(i, n) + i + 1;
    }
        pi[p] = (int32_t)i;
        pj[p] = (int32_t)j;
        const int64_t m = lens[i], c = lens[j];
        rows1[p] = m + 1;  // output rows: the first sequence's
        int cb = (int)(log2((double)(m * c)) * 2.0);
        cb = cb < 0 ? 0 : (cb >= kCostBins ? kCostBins - 1 : cb);
        // the class follows the rows the pair is swept with
        kk = pair_class((int)(tr && tr[p] ? c : m), map) * kCostBins + cb;
        key[p] = kk;
    }
    wave_count_add(hist, kk, p < P);
}

// exclusive offsets of the cost classes, most expensive class first
__global__ void k_bins(const int* __restrict__ hist, int* __restrict__ bin_start) {
    __shared__ int part[kKeyBins];
    const int t = threadIdx.x;  // kKeyBins threads
    part[t] = hist[kKeyBins - 1 - t];
    __syncthreads();
    for (int d = 1; d < kKeyBins; d <<= 1) {
        int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    bin_start[kKeyBins - 1 - t] = part[t] - hist[kKeyBins - 1 - t];
}

__global__ void k_fill_queue(int64_t P, const int32_t* __restrict__ key, const int* __restrict__ bin_start,
                             int* __restrict__ bin_fill, int32_t* __restrict__ queue) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < P;
    const int kk = valid ? key[p] : 0;
    const int rank = wave_count_add(bin_fill, kk, valid);
    if (valid) queue[bin_start[kk] + rank] = (int32_t)p;
}

// ------------------------------------------------------ int64 scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__global__ void k_scan_local(int64_t* __restrict__ d, int64_t n, int64_t* __restrict__ sums) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)t * kScanItems;
    int64_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t idx = base + q;
        const int64_t x = idx < n ? d[idx] : 0;
        v[q] = acc;
        acc += x;
    }
    part[t] = acc;
    __syncthreads();
    for (int s = 1; s < kScanThreads; s <<= 1) {
        int64_t add = t >= s ? part[t - s] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    const int64_t off = part[t] - acc;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t idx = base + q;
        if (idx < n) d[idx] = v[q] + off;
    }
    if (t == kScanThreads - 1) sums[blockIdx.x] = part[t];
}

__global__ void k_scan_add(int64_t* __restrict__ d, int64_t n, const int64_t* __restrict__ offs) {
    const int64_t idx = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    const int64_t o = offs[blockIdx.x];
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = idx + (int64_t)q * kScanThreads;
        if (i < n) d[i] += o;
    }
}

// ---------------------------------------------------- gather (a6 final)
__global__ void k_gather(int64_t P, const int64_t* __restrict__ nnz_off, const int64_t* __restrict__ pair_base, const int32_t* __restrict__ pool_col,
                         const float* __restrict__ pool_val, int32_t* __restrict__ col, float* __restrict__ val,
                         int64_t cap) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = w0; p < P; p += nw) {
        // nnz_off is the exclusive scan of the per-pair counts (P+1 entries)
        const int64_t dst = nnz_off[p], c = nnz_off[p + 1] - dst, src = pair_base[p];
        if (src + c > cap || dst + c > cap) continue;  // overflowed run: reported by the host
        for (int64_t e = lane; e < c; e += kWave) {
            col[dst + e] = pool_col[src + e];
            val[dst + e] = pool_val[src + e];
        }
    }
}

// ================================================================ host side
hipError_t launch_tables(const DevParams* p, void* tab, DevConsts* c, void* col0, int rows, int fp64, hipStream_t s) {
    int blocks = 1 + (rows + 255) / 256;
    if (blocks > 65) blocks = 65;
    if (fp64)
        hipLaunchKernelGGL(k_tables<double>, dim3(blocks), dim3(256), 0, s, p, reinterpret_cast<double2*>(tab), c,
                           reinterpret_cast<Col0*>(col0), rows);
    else
        hipLaunchKernelGGL(k_tables<float>, dim3(blocks), dim3(256), 0, s, p, reinterpret_cast<float2*>(tab), c,
                           reinterpret_cast<Col0*>(col0), rows);
    return hipGetLastError();
}

hipError_t launch_reset(int* ints, int n, hipStream_t s) {
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_reset, dim3(blocks > 1024 ? 1024 : blocks), dim3(256), 0, s, ints, n);
    return hipGetLastError();
}

hipError_t launch_setup(int32_t n, const int32_t* lens, const int32_t* list_i, const int32_t* list_j,
                        const uint8_t* tr, int64_t P,
                        int32_t* pi, int32_t* pj, int64_t* rows1, int32_t* key, int* hist, int64_t* pair_nnz,
                        const ClassMap& map, hipStream_t s) {
    const int64_t blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, n, lens, list_i, list_j,
                       tr, P, pi, pj, rows1, key, hist, pair_nnz, map);
    return hipGetLastError();
}

hipError_t launch_stage_seqs(int32_t n, int32_t alphabet, const uint8_t* seqs, const int64_t* seq_off,
                             const int32_t* lens, const int64_t* seqa_off, uint8_t* seqa, int* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = n < 2048 ? n : 2048;
    hipLaunchKernelGGL(k_stage_seqs, dim3(blocks), dim3(128), 0, s, n, alphabet, seqs, seq_off, lens, seqa_off, seqa,
                       flags);
    return hipGetLastError();
}

hipError_t launch_bins(const int* hist, int* bin_start, hipStream_t s) {
    hipLaunchKernelGGL(k_bins, dim3(1), dim3(kKeyBins), 0, s, hist, bin_start);
    return hipGetLastError();
}

hipError_t launch_fill_queue(int64_t P, const int32_t* key, const int* bin_start, int* bin_fill, int32_t* queue,
                             hipStream_t s) {
    const int64_t blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_fill_queue, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, P, key, bin_start,
                       bin_fill, queue);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
        tot += nb + 1;
        n = nb;
    }
    return tot + 1;
}

hipError_t scan_i64(int64_t* d, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d, n, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = scan_i64(tmp, nb, tmp + nb + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d, n, tmp);
    return hipGetLastError();
}

template <int R, bool MULTI>
static hipError_t launch_pairs_r(int fp64, int grid, const PairArgs& a, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL((k_pairs<R, double, MULTI>), dim3(grid), dim3(kWave * kWavesPerBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_pairs<R, float, MULTI>), dim3(grid), dim3(kWave * kWavesPerBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pairs(int cls, int fp64, int grid, const PairArgs& a, hipStream_t s) {
    switch (cls) {
        case 0: return launch_pairs_r<1, false>(fp64, grid, a, s);
        case 1: return launch_pairs_r<2, false>(fp64, grid, a, s);
        case 2: return launch_pairs_r<3, false>(fp64, grid, a, s);
        case 3: return launch_pairs_r<4, false>(fp64, grid, a, s);
        case 4: return launch_pairs_r<5, false>(fp64, grid, a, s);
        case 5: return launch_pairs_r<6, false>(fp64, grid, a, s);
        case 6: return launch_pairs_r<7, false>(fp64, grid, a, s);
        case 7: return launch_pairs_r<8, false>(fp64, grid, a, s);
        case kBandClass + 0: return launch_pairs_r<5, true>(fp64, grid, a, s);
        case kBandClass + 1: return launch_pairs_r<6, true>(fp64, grid, a, s);
        case kBandClass + 2: return launch_pairs_r<7, true>(fp64, grid, a, s);
        default: return launch_pairs_r<8, true>(fp64, grid, a, s);
    }
}

template <int R, bool MULTI>
static hipError_t launch_pair_one_r(int fp64, int64_t p, const PairArgs& a, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL((k_pair_one<R, double, MULTI>), dim3(1), dim3(kWave), 0, s, a, p);
    else
        hipLaunchKernelGGL((k_pair_one<R, float, MULTI>), dim3(1), dim3(kWave), 0, s, a, p);
    return hipGetLastError();
}

hipError_t launch_pair_one(int cls, int fp64, int64_t p, const PairArgs& a, hipStream_t s) {
    switch (cls) {
        case 0: return launch_pair_one_r<1, false>(fp64, p, a, s);
        case 1: return launch_pair_one_r<2, false>(fp64, p, a, s);
        case 2: return launch_pair_one_r<3, false>(fp64, p, a, s);
        case 3: return launch_pair_one_r<4, false>(fp64, p, a, s);
        case 4: return launch_pair_one_r<5, false>(fp64, p, a, s);
        case 5: return launch_pair_one_r<6, false>(fp64, p, a, s);
        case 6: return launch_pair_one_r<7, false>(fp64, p, a, s);
        case 7: return launch_pair_one_r<8, false>(fp64, p, a, s);
        case kBandClass + 0: return launch_pair_one_r<5, true>(fp64, p, a, s);
        case kBandClass + 1: return launch_pair_one_r<6, true>(fp64, p, a, s);
        case kBandClass + 2: return launch_pair_one_r<7, true>(fp64, p, a, s);
        default: return launch_pair_one_r<8, true>(fp64, p, a, s);
    }
}

template <int R, bool MULTI>
static hipError_t launch_pairs_ck_r(int grid, const PairArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_pairs_ck<R, MULTI>), dim3(grid), dim3(kWave * kWavesPerBlock), 0, s, a);
    return hipGetLastError();
}

// The checkpointed form exists for classes of 1..kCkMaxRows rows per lane:
// beyond that the routine does not fit the registers, the compiler stops
// inlining it into the kernel (a called function, its arguments through a
// stack in scratch memory) and such a kernel faulted the GPU with the cause
// not identified, so it is not built.
hipError_t launch_pairs_ck(int cls, int grid, const PairArgs& a, hipStream_t s) {
    switch (cls) {
        case 0: return launch_pairs_ck_r<1, false>(grid, a, s);
        case 1: return launch_pairs_ck_r<2, false>(grid, a, s);
        case 2: return launch_pairs_ck_r<3, false>(grid, a, s);
        case 3: return launch_pairs_ck_r<4, false>(grid, a, s);
        case 4: return launch_pairs_ck_r<5, false>(grid, a, s);
        default: return class_banded(cls) ? launch_pairs_ck_r<kCkBandRows, true>(grid, a, s) : hipErrorInvalidValue;
    }
}

template <int R, bool MULTI>
static hipError_t launch_pair_one_ck_r(int64_t p, const PairArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_pair_one_ck<R, MULTI>), dim3(1), dim3(kWave), 0, s, a, p);
    return hipGetLastError();
}

hipError_t launch_pair_one_ck(int cls, int64_t p, const PairArgs& a, hipStream_t s) {
    switch (cls) {
        case 0: return launch_pair_one_ck_r<1, false>(p, a, s);
        case 1: return launch_pair_one_ck_r<2, false>(p, a, s);
        case 2: return launch_pair_one_ck_r<3, false>(p, a, s);
        case 3: return launch_pair_one_ck_r<4, false>(p, a, s);
        case 4: return launch_pair_one_ck_r<5, false>(p, a, s);
        default: return class_banded(cls) ? launch_pair_one_ck_r<kCkBandRows, true>(p, a, s) : hipErrorInvalidValue;
    }
}

template <int R, bool MULTI>
static int blocks_per_cu_ck_r() {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pairs_ck<R, MULTI>,
                                                                kWave * kWavesPerBlock, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

int pairs_ck_blocks_per_cu(int cls) {
    switch (cls) {
        case 0: return blocks_per_cu_ck_r<1, false>();
        case 1: return blocks_per_cu_ck_r<2, false>();
        case 2: return blocks_per_cu_ck_r<3, false>();
        case 3: return blocks_per_cu_ck_r<4, false>();
        case 4: return blocks_per_cu_ck_r<5, false>();
        default: return class_banded(cls) ? blocks_per_cu_ck_r<kCkBandRows, true>() : 1;
    }
}

int ck_state_words(int R) { return ck_words(R); }

template <int R, bool MULTI>
static int blocks_per_cu_r(int fp64) {
    int nb = 0;
    hipError_t e;
    if (fp64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pairs<R, double, MULTI>,
                                                         kWave * kWavesPerBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pairs<R, float, MULTI>,
                                                         kWave * kWavesPerBlock, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

int pairs_blocks_per_cu(int cls, int fp64) {
    switch (cls) {
        case 0: return blocks_per_cu_r<1, false>(fp64);
        case 1: return blocks_per_cu_r<2, false>(fp64);
        case 2: return blocks_per_cu_r<3, false>(fp64);
        case 3: return blocks_per_cu_r<4, false>(fp64);
        case 4: return blocks_per_cu_r<5, false>(fp64);
        case 5: return blocks_per_cu_r<6, false>(fp64);
        case 6: return blocks_per_cu_r<7, false>(fp64);
        case 7: return blocks_per_cu_r<8, false>(fp64);
        case kBandClass + 0: return blocks_per_cu_r<5, true>(fp64);
        case kBandClass + 1: return blocks_per_cu_r<6, true>(fp64);
        case kBandClass + 2: return blocks_per_cu_r<7, true>(fp64);
        default: return blocks_per_cu_r<8, true>(fp64);
    }
}

size_t col0_bytes() { return sizeof(Col0); }
size_t fwd_bnd_bytes(int fp64) { return fp64 ? sizeof(FwdBnd<double>) : sizeof(FwdBnd<float>); }
size_t bwd_bnd_bytes(int fp64) { return fp64 ? sizeof(BwdBnd<double>) : sizeof(BwdBnd<float>); }

hipError_t launch_gather(int64_t P, const int64_t* nnz_off, const int64_t* pair_base,
                         const int32_t* pool_col, const float* pool_val, int32_t* col, float* val, int64_t cap,
                         hipStream_t s) {
    int64_t blocks = (P + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, s, P, nnz_off, pair_base, pool_col,
                       pool_val, col, val, cap);
    return hipGetLastError();
}

}  // namespace qp
