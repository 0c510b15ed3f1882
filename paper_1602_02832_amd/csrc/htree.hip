// Block-step force evaluation of the tree/Hermite scheme on gfx950 (CDNA4).
//
// Fukushige & Kawai, Section 2: at each block step the j-memory (particles
// and tree nodes as pseudo-particles) is predicted to the block time and the
// force, its time derivative and the potential on every active particle are
// summed over the interaction list of the particle's group.  The paper does
// this with GRAPE-9 FPGA pipelines fed by an indirect addressing unit; here
// it is one HIP kernel over work items (group, i-tile, list range):
//
//  * A work-group of 256 threads (four wave64) holds an i-tile of T active
//    particles of one group (T a power of two, 1..256) and splits the list
//    into S = 256 / T j-streams: thread t owns i-slot t % T and j-stream t / T.
//  * The list range is walked in rounds of 256 entries.  In each round every
//    thread gathers one entry of the combined memory, predicts it to the
//    block time in registers (or reads the eagerly predicted arrays) and
//    stages it in LDS; then every thread sums its i against its j-stream's
//    share of the round.  For T >= 64 all lanes of a wave read the same
//    entry, which LDS broadcasts.
//  * Partial sums of the S j-streams are reduced through LDS in a fixed order.
//    Long lists of small tiles are split over several items (more parallel
//    work for sparse block steps); their partials are summed in split order
//    by a second kernel, so results never depend on scheduling.
//
// The pair sum is not a dense contraction (one rsqrt per pair), so it runs
// on the vector ALUs; no matrix-core instructions are used.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "htree.h"
#include "htree_tree.h"
#include "wave_ops.h"

namespace {

// ------------------------------------------------------------------------------------------------
// errors
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HT_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(HT_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------------------------------------
// device data structures
constexpr int kWG = 256;      // threads per work-group
constexpr int kRound = 256;   // list entries staged per round and entry multiple (one per thread)
// Small tiles give a thread few pairs per staged entry, so their rounds are
// latency-bound: for T <= 8 every thread gathers two entries per round.
__host__ __device__ constexpr int round_mult(int T) { return T <= 8 ? 2 : 1; }
constexpr int kRoundMax = 2 * kRound;
constexpr int kOut = 7;       // acc[3], jerk[3], pot
constexpr int kMaxBatch = 1024;   // clusters per batched launch

// j-memory record of one particle or node: everything the predictor needs in
// one 128-byte line, so a list-indexed gather touches a single cache line
// (lists reach nodes in scattered order; a field-per-array layout would touch
// one line per field).
struct alignas(128) RecFp64 {
    double x, y, z, t0;
    double vx, vy, vz, m;
    double ax, ay, az, pad0;
    double jx, jy, jz, pad1;
};
struct alignas(128) RecMixed {
    double x, y, z, t0;
    double vx, vy, vz;
    float m, ax, ay, az, jx, jy, jz;
    float pad[9];
};
// Eagerly predicted state (EAGER mode): 64 bytes per entry.
struct alignas(64) PRecFp64 {
    double x, y, z, m;
    double vx, vy, vz, pad;
};
struct alignas(64) PRecMixed {
    double x, y, z;
    double vx, vy, vz;
    float m, pad0;
    double pad1;
};
static_assert(sizeof(RecFp64) == 128 && sizeof(RecMixed) == 128, "record size");
static_assert(sizeof(PRecFp64) == 64 && sizeof(PRecMixed) == 64, "predicted record size");

// Everything a kernel needs to know about one cluster (context) for one call.
struct Desc {
    const void* rec;    // [N+M] raw records (RecFp64 or RecMixed)
    void* prec;         // [N+M] predicted records (EAGER mode)
    const int32_t* entries;
    const int32_t* active;
    double* acc;        // [n_active][3]
    double* jerk;       // [n_active][3]
    double* pot;        // [n_active]
    double* partial;    // split partial sums, kOut doubles per slot
    double t;
    double eps2;
    // run-length lists (HT_LISTS_RUNS): run r covers list positions
    // run_pos[r] .. run_pos[r+1]-1 with the combined indices run_start[r],
    // run_start[r]+1, ...; indices from copy_base on are the groups' node copies
    // (copy_rec[index - copy_base]); item_runs[k] is the run holding item k's
    // first position
    const int32_t* run_start;
    const int64_t* run_pos;
    const int64_t* item_runs;
    const void* copy_rec;
    int64_t n_runs;
    int32_t copy_base;
    // 1: eps2 > 0 and every list holds each particle of its group exactly once
    // (direct sums: every particle once), so the pair loop sums the self pair
    // too, which adds exactly zero to acc and jerk, and the items that carry
    // kSelfTerm take its potential term -m_i / eps back (no per-pair test)
    int32_t self_once;
    // union tiles (HT_LISTS_UNION): the union lists of runs of consecutive
    // groups (entries) with a bit per member group whose own list holds the
    // entry (mask); the member index of each active position (act_member)
    const int32_t* u_entries;
    const uint8_t* u_mask;
    const uint8_t* act_member;
};

// One unit of work: an i-tile of one group against a range of its list.
struct Item {
    int64_t j_begin;    // first list entry (or first particle, direct sum)
    int64_t j_end;
    int64_t out;        // -1: final results; otherwise partial slot of i-slot 0
    int32_t act_begin;  // active-array position of i-slot 0
    int16_t n_i;        // valid i-slots (1..T)
    int16_t tile_log2;  // T = 1 << (tile_log2 & kTileMask); kSelfTerm: the item holding the start of its
                        // tile's list range, which takes the self pair's potential back; kUnion: the
                        // range is in the union lists, and a pair counts only where the entry's mask
                        // holds the i-slot's member bit
};
constexpr int16_t kTileMask = 0xff;
constexpr int16_t kSelfTerm = 0x100;
constexpr int16_t kUnion = 0x200;

// The partial sums of one split i-tile: nsplit blocks of n_i slots.
struct RTile {
    int64_t pbase;
    int32_t act_begin;
    int32_t n_i;
    int32_t nsplit;
    int32_t pad;
};

// One cluster in a launch: its descriptor and where its items sit in the
// launch's global item numbering.
struct Entry {
    Desc d;
    const Item* items;
    const RTile* rtiles;
    int64_t first_item;
    int64_t first_rtile;
    int64_t n_items;    // entry 0: items and split tiles of the whole launch (graph replays
    int64_t n_rtiles;   // read them here, their launch arguments being fixed)
};

struct PrecFp64 {
    using Stored = double;  // stored a, jerk, m
    using Vel = double;     // predicted velocity used in the pair
    using Rec = RecFp64;
    using PRec = PRecFp64;
    static constexpr bool kMixed = false;
};
struct PrecMixed {
    using Stored = float;
    using Vel = double;
    using Rec = RecMixed;
    using PRec = PRecMixed;
    static constexpr bool kMixed = true;
};

// One staged j of a round: predicted position and velocity, mass (widened
// once at staging), combined index.  Records (not one array per field) so
// that a thread reads an entry with a few 16-byte LDS loads at immediate
// offsets from one address.
template <class P>
struct alignas(16) JRec {
    double x, y, z;
    typename P::Vel vx, vy, vz;
    double m;
    int32_t idx;
    int32_t mask;   // union tiles: the member groups whose lists hold the entry
};
static_assert(sizeof(JRec<PrecMixed>) == 64 && sizeof(JRec<PrecFp64>) == 64, "staged records are 64 bytes");

template <class P>
union LdsAll {
    JRec<P> j[kRoundMax];
    double red[kOut * kWG];
};

// Run-length lists: the runs that overlap a round, as (first position in the
// round, index at position 0 of the round).
struct RunLds {
    int32_t pos[kRoundMax];
    int32_t off[kRoundMax];
};
struct NoRunLds {};

// ------------------------------------------------------------------------------------------------
// predictor (4th-order Hermite, Section 1/2): Taylor series to the jerk, FP64.
template <class P>
__device__ __forceinline__ void predict_rec(const typename P::Rec& r, double t, double& x, double& y, double& z,
                                            double& vx, double& vy, double& vz) {
    const double dt = t - r.t0;
    const double h2 = 0.5 * dt, h3 = dt * (1.0 / 3.0);
    const double a0 = static_cast<double>(r.ax), a1 = static_cast<double>(r.ay), a2 = static_cast<double>(r.az);
    const double j0 = static_cast<double>(r.jx), j1 = static_cast<double>(r.jy), j2 = static_cast<double>(r.jz);
    x = r.x + dt * (r.vx + h2 * (a0 + h3 * j0));
    y = r.y + dt * (r.vy + h2 * (a1 + h3 * j1));
    z = r.z + dt * (r.vz + h2 * (a2 + h3 * j2));
    vx = r.vx + dt * (a0 + h2 * j0);
    vy = r.vy + dt * (a1 + h2 * j1);
    vz = r.vz + dt * (a2 + h2 * j2);
}

// Position, velocity (in the pair's precision) and mass of entry j at the block time.
// RUNS: indices from copy_base on are node copies, in their own array.
template <class P, bool EAGER, bool RUNS = false>
__device__ __forceinline__ void load_state(const Desc& c, int j, double& x, double& y, double& z,
                                           typename P::Vel& vx, typename P::Vel& vy, typename P::Vel& vz,
                                           typename P::Stored& m) {
    using V = typename P::Vel;
    if constexpr (EAGER) {
        const typename P::PRec r = static_cast<const typename P::PRec*>(c.prec)[j];
        x = r.x;
        y = r.y;
        z = r.z;
        vx = r.vx;
        vy = r.vy;
        vz = r.vz;
        m = r.m;
    } else {
        const typename P::Rec* base = static_cast<const typename P::Rec*>(c.rec);
        if constexpr (RUNS) {
            if (j >= c.copy_base) base = static_cast<const typename P::Rec*>(c.copy_rec) - c.copy_base;
        }
        const typename P::Rec r = base[j];
        double dvx, dvy, dvz;
        predict_rec<P>(r, c.t, x, y, z, dvx, dvy, dvz);
        vx = static_cast<V>(dvx);
        vy = static_cast<V>(dvy);
        vz = static_cast<V>(dvz);
        m = r.m;
    }
}

// ------------------------------------------------------------------------------------------------
// pair interaction: r = x_j - x_i, w = v_j - v_i, s = r.r + eps^2
//   a += m r s^-3/2,  jerk += m s^-3/2 (w - 3 (r.w)/s r),  pot -= m s^-1/2
struct Acc64 {
    double v[kOut];
};

// SKIP: the self pair (J.idx == i) is masked out; otherwise it is summed
// like any other pair (see Desc::self_once).
// MASK (union tiles): the pair counts only where the entry's member mask
// holds bit mb, the i-particle's group within the run.
template <bool SKIP, bool MASK>
__device__ __forceinline__ void pair_fp64(double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                          int i, const JRec<PrecFp64>& J, double eps2, Acc64& A, int mb) {
    const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
    const double wx = J.vx - vxi, wy = J.vy - vyi, wz = J.vz - vzi;
    const double s = dx * dx + dy * dy + dz * dz + eps2;
    double rinv = rsqrt(s);
    if constexpr (SKIP) rinv = (J.idx == i) ? 0.0 : rinv;
    if constexpr (MASK) rinv = ((J.mask >> mb) & 1) ? rinv : 0.0;
    const double rinv2 = rinv * rinv;
    const double mr = J.m * rinv;
    const double mr3 = mr * rinv2;
    const double alpha = 3.0 * (dx * wx + dy * wy + dz * wz) * rinv2;
    A.v[0] += mr3 * dx;
    A.v[1] += mr3 * dy;
    A.v[2] += mr3 * dz;
    A.v[3] += mr3 * (wx - alpha * dx);
    A.v[4] += mr3 * (wy - alpha * dy);
    A.v[5] += mr3 * (wz - alpha * dz);
    A.v[6] -= mr;
}

// Mixed form: the j-memory stores m, a and jerk in FP32 (the predictor reads
// them), and s^-1/2 starts from the FP32 reciprocal square root (v_rsq_f32,
// about one ulp) refined by one Newton step in FP64 in residual form
// (e = 1 - s y^2, y += y e / 2), which leaves a relative error near 1e-13.
// Everything else is FP64.  The jerk is a sum of terms that can cancel to a
// few hundredths of their magnitudes; with s^-3/2 and the jerk terms in FP32
// (a few ulp each) such particles missed the 1e-5 jerk target, so only the
// seed is FP32.  FP64 FMAs issue at the non-packed FP32 rate on this chip.
template <bool SKIP, bool MASK>
__device__ __forceinline__ void pair_mixed(double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                           int i, const JRec<PrecMixed>& J, double eps2, Acc64& A, int mb) {
    const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
    const double s = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
    const double y0 = static_cast<double>(__builtin_amdgcn_rsqf(static_cast<float>(s)));
    const double e = fma(-(s * y0), y0, 1.0);
    double rinv = fma(0.5 * y0, e, y0);
    if constexpr (SKIP) rinv = (J.idx == i) ? 0.0 : rinv;
    if constexpr (MASK) rinv = ((J.mask >> mb) & 1) ? rinv : 0.0;
    const double rinv2 = rinv * rinv;
    const double mr = J.m * rinv;
    const double mr3 = mr * rinv2;
    const double wx = J.vx - vxi, wy = J.vy - vyi, wz = J.vz - vzi;
    const double alpha = 3.0 * fma(dz, wz, fma(dy, wy, dx * wx)) * rinv2;
    A.v[0] = fma(mr3, dx, A.v[0]);
    A.v[1] = fma(mr3, dy, A.v[1]);
    A.v[2] = fma(mr3, dz, A.v[2]);
    A.v[3] = fma(mr3, fma(-alpha, dx, wx), A.v[3]);
    A.v[4] = fma(mr3, fma(-alpha, dy, wy), A.v[4]);
    A.v[5] = fma(mr3, fma(-alpha, dz, wz), A.v[5]);
    A.v[6] -= mr;
}

template <class P, bool SKIP = true, bool MASK = false>
__device__ __forceinline__ void pair(double xi, double yi, double zi, double vxi, double vyi, double vzi, int i,
                                     const JRec<P>& J, double eps2, Acc64& A, int mb = 0) {
    if constexpr (P::kMixed) pair_mixed<SKIP, MASK>(xi, yi, zi, vxi, vyi, vzi, i, J, eps2, A, mb);
    else pair_fp64<SKIP, MASK>(xi, yi, zi, vxi, vyi, vzi, i, J, eps2, A, mb);
}

// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void write_out(const Desc& c, int64_t o, const double* v) {
    c.acc[3 * o + 0] = v[0];
    c.acc[3 * o + 1] = v[1];
    c.acc[3 * o + 2] = v[2];
    c.jerk[3 * o + 0] = v[3];
    c.jerk[3 * o + 1] = v[4];
    c.jerk[3 * o + 2] = v[5];
    c.pot[o] = v[6];
}

// ------------------------------------------------------------------------------------------------
// one work item with tile size T
template <class P, bool EAGER, bool DIRECT, bool RUNS, int T, class RL, bool UNI = false>
__device__ __forceinline__ void run_item(const Desc& c, const Item& it, int64_t run0, LdsAll<P>& lds, RL& rl) {
    constexpr int G = round_mult(T);    // entries gathered per thread and round
    constexpr int R = kRound * G;       // entries per round
    constexpr int S = kWG / T;          // j-streams
    constexpr int PER = R / S;          // pairs per thread in a full round (= G T)
    const int tid = threadIdx.x;
    const int islot = tid & (T - 1);
    const int stream = tid / T;
    const bool has_i = islot < it.n_i;
    // List indices of the round about to be gathered, loaded one round ahead so
    // that a round's gather waits on one memory access (the record) instead of
    // two in a row (index, then record); the first round's are loaded beside
    // the i-particle's own record.
    // Union tiles read the run's union list and each entry's member mask.
    const bool uni = UNI && (it.tile_log2 & kUnion);
    const int32_t* ent = uni ? c.u_entries : c.entries;
    int jn[G];
    auto load_idx = [&](int64_t b) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t e = b + tid + g * kWG;
            jn[g] = e < it.j_end ? (DIRECT ? static_cast<int>(e) : ent[e]) : 0;
        }
    };
    // Run-length lists: the round's indices are expanded from its runs after the
    // round's first barrier (run: the run holding the round's first position).
    int64_t run = run0;
    if constexpr (!RUNS) load_idx(it.j_begin);
    const int i = c.active[it.act_begin + (has_i ? islot : 0)];
    const int mb = uni ? static_cast<int>(c.act_member[it.act_begin + (has_i ? islot : 0)]) : 0;

    double xi, yi, zi;
    typename P::Vel vxi, vyi, vzi;
    typename P::Stored mi;
    load_state<P, EAGER>(c, i, xi, yi, zi, vxi, vyi, vzi, mi);

    Acc64 A;
#pragma unroll
    for (int q = 0; q < kOut; ++q) A.v[q] = 0.0;

    for (int64_t base = it.j_begin; base < it.j_end; base += R) {
        const int64_t rest = it.j_end - base;
        const int cnt = rest < R ? static_cast<int>(rest) : R;
        __syncthreads();  // the previous round is no longer read
        if constexpr (RUNS) {
            // the runs overlapping [base, base + cnt) are run, run + 1, ...: at most cnt
            int ov = 0;
            for (int k = tid; k < cnt; k += kWG) {
                const int64_t q = run + k;
                if (q < c.n_runs) {
                    const int64_t p = c.run_pos[q];
                    if (p < base + cnt) {
                        const int64_t p0 = p > base ? p : base;
                        rl.pos[k] = static_cast<int32_t>(p0 - base);
                        rl.off[k] = static_cast<int32_t>(c.run_start[q] + (p0 - p) - (p0 - base));
                        ++ov;
                    }
                }
            }
            const int nr = __syncthreads_count(ov);   // the loaded runs are visible from here on
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int e = tid + g * kWG;
                if (e < cnt) {   // the last loaded run starting at or before e
                    int lo = 0, hi = nr;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (rl.pos[mid] <= e) lo = mid; else hi = mid;
                    }
                    jn[g] = rl.off[lo] + e;
                }
            }
            // the run holding the next round's first position
            const int64_t nx = run + nr < c.n_runs ? c.run_pos[run + nr] : INT64_MAX;
            run += nx == base + cnt ? nr : nr - 1;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int e = tid + g * kWG;
            if (e < cnt) {
                const int j = jn[g];
                double xj, yj, zj;
                typename P::Vel vxj, vyj, vzj;
                typename P::Stored mj;
                load_state<P, EAGER, RUNS>(c, j, xj, yj, zj, vxj, vyj, vzj, mj);
                if constexpr (UNI) {   // the mask is loaded beside the record
                    const int mask = uni ? static_cast<int>(c.u_mask[base + e]) : 0;
                    lds.j[e] = JRec<P>{xj, yj, zj, vxj, vyj, vzj, static_cast<double>(mj), j, mask};
                } else {   // the mask word is never read
                    JRec<P>& r = lds.j[e];
                    r.x = xj;
                    r.y = yj;
                    r.z = zj;
                    r.vx = vxj;
                    r.vy = vyj;
                    r.vz = vzj;
                    r.m = static_cast<double>(mj);
                    r.idx = j;
                }
            }
        }
        if constexpr (!RUNS) {
            if (base + R < it.j_end) load_idx(base + R);   // in flight during this round's pairs
        }
        __syncthreads();
        const double eps2 = c.eps2;
        // the round's pairs: SK masks the self pair (not needed when every list
        // holds each particle once), MK masks entries outside the i-particle's
        // own list (union tiles)
        auto pairs_of_round = [&](auto sk, auto mkt) {
            constexpr bool SK = decltype(sk)::value, MK = decltype(mkt)::value;
            if (cnt == R) {
#pragma unroll 4
                for (int u = 0; u < PER; ++u)
                    pair<P, SK, MK>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[stream + u * S], eps2, A, mb);
            } else {
#pragma unroll 1
                for (int k = stream; k < cnt; k += S)
                    pair<P, SK, MK>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[k], eps2, A, mb);
            }
        };
        using Yes = std::true_type;
        using No = std::false_type;
        if constexpr (UNI) {
            if (uni) {
                if (c.self_once) pairs_of_round(No{}, Yes{});
                else pairs_of_round(Yes{}, Yes{});
            } else {
                if (c.self_once) pairs_of_round(No{}, No{});
                else pairs_of_round(Yes{}, No{});
            }
        } else if (c.self_once) {
            if (cnt == R) {
#pragma unroll 4
                for (int u = 0; u < PER; ++u)
                    pair<P, false>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[stream + u * S], eps2, A);
            } else {
#pragma unroll 1
                for (int k = stream; k < cnt; k += S) pair<P, false>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[k], eps2, A);
            }
        } else {
            if (cnt == R) {
#pragma unroll 4
                for (int u = 0; u < PER; ++u) pair<P>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[stream + u * S], eps2, A);
            } else {
#pragma unroll 1
                for (int k = stream; k < cnt; k += S) pair<P>(xi, yi, zi, vxi, vyi, vzi, i, lds.j[k], eps2, A);
            }
        }
    }

    // Reduce the S j-streams of each i-slot in a fixed order, so results never
    // depend on timing.  T < 64: the 64 / T streams of a wave first, by a
    // pairwise tree of lane exchanges (stream s += stream s + h, h = 32/T, ...,
    // 1, i.e. lane offsets 32 down to T), then the four waves in order through
    // LDS.  T >= 64 (at most four streams, whole waves each): a pairwise tree
    // in LDS.
    if constexpr (T < 64) {
        auto add = [](double p, double q) { return p + q; };
#pragma unroll
        for (int q = 0; q < kOut; ++q) A.v[q] = wave_ops::tree<32, T>(A.v[q], add);
        const int lane = tid & 63, wave = tid >> 6;
        __syncthreads();
        if (lane < T) {
#pragma unroll
            for (int q = 0; q < kOut; ++q) lds.red[q * kWG + wave * T + lane] = A.v[q];
        }
        __syncthreads();
        if (tid < T) {
#pragma unroll
            for (int q = 0; q < kOut; ++q)
                A.v[q] = ((lds.red[q * kWG + islot] + lds.red[q * kWG + T + islot]) + lds.red[q * kWG + 2 * T + islot]) +
                         lds.red[q * kWG + 3 * T + islot];
        }
    } else if constexpr (S > 1) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kOut; ++q) lds.red[q * kWG + tid] = A.v[q];
#pragma unroll
        for (int h = S / 2; h >= 1; h /= 2) {
            __syncthreads();
            if (stream < h) {
#pragma unroll
                for (int q = 0; q < kOut; ++q) lds.red[q * kWG + tid] += lds.red[q * kWG + tid + h * T];
            }
        }
        __syncthreads();
        if (stream == 0) {
#pragma unroll
            for (int q = 0; q < kOut; ++q) A.v[q] = lds.red[q * kWG + islot];
        }
    }
    if (stream == 0 && has_i) {
        if (c.self_once && (it.tile_log2 & kSelfTerm)) {
            // the self pair's potential term, as the pair loop summed it (same
            // inputs, same operations; its acc and jerk terms are exact zeros)
            Acc64 Z;
#pragma unroll
            for (int q = 0; q < kOut; ++q) Z.v[q] = 0.0;
            pair<P, false>(xi, yi, zi, vxi, vyi, vzi, i,
                           JRec<P>{xi, yi, zi, vxi, vyi, vzi, static_cast<double>(mi), i, 0}, c.eps2, Z);
            A.v[6] -= Z.v[6];
        }
        if (it.out < 0) {
            write_out(c, it.act_begin + islot, A.v);
        } else {
            double* p = c.partial + (it.out + islot) * kOut;
#pragma unroll
            for (int q = 0; q < kOut; ++q) p[q] = A.v[q];
        }
    }
}

__device__ __forceinline__ int find_entry(const Entry* tab, int n_tab, int64_t g, bool rtile) {
    int lo = 0, hi = n_tab;  // first_* of tab[lo] <= g < first_* of tab[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const int64_t f = rtile ? tab[mid].first_rtile : tab[mid].first_item;
        if (f <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Register budget: the mixed form fits 128 VGPRs (4 waves per SIMD) without
// spilling; the FP64 form, the run-length lists' expansion and the union
// tiles' masked pairs need a little more and run 3 waves per SIMD.
template <class P, bool RUNS = false, bool UNI = false>
struct WavesPerSimd { static constexpr int value = P::kMixed && !RUNS && !UNI ? 4 : 3; };

// Work-group g takes items g, g + grid, ...  The grid is normally the item
// count; graph replays and device loops launch a fixed grid and pass
// n_items < 0, and the count is read from counts[0] (the items of the whole
// launch, written by the plan's delivery or by the device planner).  (A shared atomic work counter was measured to cost
// about 1 us per item: device-scope atomics on one address serialise across
// the eight XCDs.)
// Placed plans (bins != nullptr): the items come in n_bins runs, run x being
// items bins[x] .. bins[x+1]-1, and work-group b takes the items of run
// b % n_bins from position b / n_bins on, in steps of grid / n_bins (the grid
// is n_bins times the longest run).  Work-groups are handed to the XCDs in
// turn, so each run stays on one XCD and its L2.
// UNI: the plan holds union-tile items (a separate instantiation, so that the
// plain kernel keeps its register budget).
template <class P, bool EAGER, bool DIRECT, bool RUNS = false, bool UNI = false>
__global__ __launch_bounds__(kWG, (WavesPerSimd<P, RUNS, UNI>::value)) void force_kernel(const Entry* __restrict__ tab,
                                                                                   int n_tab, int64_t n_items,
                                                                                   const int64_t* counts,
                                                                                   const int64_t* bins = nullptr,
                                                                                   int n_bins = 1) {
    __shared__ LdsAll<P> lds;
    __shared__ typename std::conditional<RUNS, RunLds, NoRunLds>::type rl;
    if (n_items < 0) n_items = counts[0];
    int64_t g0 = blockIdx.x, step = gridDim.x;
    if (bins) {
        const int x = static_cast<int>(blockIdx.x % static_cast<unsigned>(n_bins));
        g0 = bins[x] + blockIdx.x / static_cast<unsigned>(n_bins);
        step = gridDim.x / static_cast<unsigned>(n_bins);
        n_items = bins[x + 1];
    }
    for (int64_t g = g0; g < n_items; g += step) {
        const int cl = find_entry(tab, n_tab, g, false);
        const Desc& c = tab[cl].d;
        const int64_t k = g - tab[cl].first_item;
        const Item it = tab[cl].items[k];
        const int64_t r0 = RUNS ? c.item_runs[k] : 0;
        switch (it.tile_log2 & kTileMask) {
            case 8: run_item<P, EAGER, DIRECT, RUNS, 256, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 7: run_item<P, EAGER, DIRECT, RUNS, 128, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 6: run_item<P, EAGER, DIRECT, RUNS, 64, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 5: run_item<P, EAGER, DIRECT, RUNS, 32, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 4: run_item<P, EAGER, DIRECT, RUNS, 16, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 3: run_item<P, EAGER, DIRECT, RUNS, 8, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 2: run_item<P, EAGER, DIRECT, RUNS, 4, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            case 1: run_item<P, EAGER, DIRECT, RUNS, 2, decltype(rl), UNI>(c, it, r0, lds, rl); break;
            default: run_item<P, EAGER, DIRECT, RUNS, 1, decltype(rl), UNI>(c, it, r0, lds, rl); break;
        }
        __syncthreads();
    }
}

// Sum the split partials of each i-slot in split order (a separate launch:
// the kernel boundary makes every partial visible, with no device-wide
// fences in the force kernel).  A tile's partials are first loaded into LDS
// by all threads at once, so the dependent adds read LDS, not memory.
constexpr int kRedLds = 6144;   // doubles of LDS for one tile's partials

// n_rtiles < 0 (graph replays): the count is read from the table.
__global__ __launch_bounds__(kWG) void reduce_kernel(const Entry* __restrict__ tab, int n_tab, int64_t n_rtiles) {
    __shared__ double buf[kRedLds];
    if (n_rtiles < 0) n_rtiles = tab[0].n_rtiles;
    for (int64_t g = blockIdx.x; g < n_rtiles; g += gridDim.x) {
        const int cl = find_entry(tab, n_tab, g, true);
        const Desc& c = tab[cl].d;
        const RTile rt = tab[cl].rtiles[g - tab[cl].first_rtile];
        const int64_t nval = static_cast<int64_t>(rt.nsplit) * rt.n_i * kOut;
        const double* src = c.partial + rt.pbase * kOut;
        if (nval <= kRedLds) {
            __syncthreads();
            for (int k = threadIdx.x; k < nval; k += kWG) buf[k] = src[k];
            __syncthreads();
        }
        for (int s = threadIdx.x; s < rt.n_i; s += kWG) {
            const double* p = nval <= kRedLds ? buf : src;
            double A[kOut];
#pragma unroll
            for (int q = 0; q < kOut; ++q) A[q] = p[static_cast<int64_t>(s) * kOut + q];
            for (int b = 1; b < rt.nsplit; ++b) {
                const double* pb = p + (static_cast<int64_t>(b) * rt.n_i + s) * kOut;
#pragma unroll
                for (int q = 0; q < kOut; ++q) A[q] += pb[q];
            }
            write_out(c, rt.act_begin + s, A);
        }
    }
}

// Predict the whole combined memory into the EAGER records.
template <class P>
__global__ __launch_bounds__(kWG) void predict_all_kernel(Desc c, int n_total) {
    using V = typename P::Vel;
    const typename P::Rec* rec = static_cast<const typename P::Rec*>(c.rec);
    typename P::PRec* prec = static_cast<typename P::PRec*>(c.prec);
    for (int j = blockIdx.x * kWG + threadIdx.x; j < n_total; j += gridDim.x * kWG) {
        const typename P::Rec r = rec[j];
        double x, y, z, vx, vy, vz;
        predict_rec<P>(r, c.t, x, y, z, vx, vy, vz);
        typename P::PRec o{};
        o.x = x;
        o.y = y;
        o.z = z;
        o.vx = static_cast<V>(vx);
        o.vy = static_cast<V>(vy);
        o.vz = static_cast<V>(vz);
        o.m = r.m;
        prec[j] = o;
    }
}

// Predicted state of selected entries, FP64 (the predictor used by the force kernels).
template <class P>
__global__ __launch_bounds__(kWG) void predict_some_kernel(Desc c, const int32_t* idx, int n, double* out_x,
                                                           double* out_v) {
    const typename P::Rec* rec = static_cast<const typename P::Rec*>(c.rec);
    for (int k = blockIdx.x * kWG + threadIdx.x; k < n; k += gridDim.x * kWG) {
        double x, y, z, vx, vy, vz;
        predict_rec<P>(rec[idx[k]], c.t, x, y, z, vx, vy, vz);
        out_x[3 * k] = x;
        out_x[3 * k + 1] = y;
        out_x[3 * k + 2] = z;
        out_v[3 * k] = vx;
        out_v[3 * k + 1] = vy;
        out_v[3 * k + 2] = vz;
    }
}

// One j-memory record from its parts (FP64 in, stored precision out).
template <class P>
__device__ __forceinline__ void store_rec(typename P::Rec* rec, int j, double t0, double m, const double* x,
                                          const double* v, const double* a, const double* jerk) {
    using S = typename P::Stored;
    typename P::Rec r{};
    r.x = x[0];
    r.y = x[1];
    r.z = x[2];
    r.t0 = t0;
    r.vx = v[0];
    r.vy = v[1];
    r.vz = v[2];
    r.m = static_cast<S>(m);
    r.ax = static_cast<S>(a[0]);
    r.ay = static_cast<S>(a[1]);
    r.az = static_cast<S>(a[2]);
    r.jx = static_cast<S>(jerk[0]);
    r.jy = static_cast<S>(jerk[1]);
    r.jz = static_cast<S>(jerk[2]);
    rec[j] = r;
}

// An update row names a particle index that is not in [0, lim): the row is
// dropped and the context's error word (pinned host memory, read by the host
// after its next synchronisation) is set.  Indices that come from device
// memory cannot be checked by the host before the launch.
__device__ __forceinline__ bool row_index_ok(int32_t j, int32_t lim, int32_t* err) {
    if (j >= 0 && j < lim) return true;
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return false;
}

// j-memory update (steps 1 and 6): rows [n][3] written into records.
// idx == nullptr: row k goes to base + k.  t0 == nullptr: every t0 = t0_all.
// idx != nullptr: rows whose index is outside [0, lim) are dropped (err set).
template <class P>
__global__ __launch_bounds__(kWG) void scatter_kernel(Desc dst, int n, const int32_t* idx, int base,
                                                      const double* t0, double t0_all, const double* m,
                                                      const double* x, const double* v, const double* a,
                                                      const double* jerk, int32_t lim, int32_t* err) {
    typename P::Rec* rec = static_cast<typename P::Rec*>(const_cast<void*>(dst.rec));
    for (int k = blockIdx.x * kWG + threadIdx.x; k < n; k += gridDim.x * kWG) {
        const int32_t j = idx ? idx[k] : base + k;
        if (idx && !row_index_ok(j, lim, err)) continue;
        store_rec<P>(rec, j, t0 ? t0[k] : t0_all, m[k], x + 3 * k, v + 3 * k, a + 3 * k, jerk + 3 * k);
    }
}

// Run-length lists: the groups' node copies, record by record (copy k is
// record idx[k] of the combined memory).
template <class P>
__global__ __launch_bounds__(kWG) void copy_records_kernel(const void* src, const int32_t* __restrict__ idx, int64_t n,
                                                           void* dst) {
    const typename P::Rec* s = static_cast<const typename P::Rec*>(src);
    typename P::Rec* d = static_cast<typename P::Rec*>(dst);
    for (int64_t k = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kWG)
        d[k] = s[idx[k]];
}

// Resident rebuild: dt and pot in the new particle order.
__global__ __launch_bounds__(kWG) void permute2_kernel(int n, const int64_t* __restrict__ perm,
                                                       const double* __restrict__ a, const double* __restrict__ b,
                                                       double* __restrict__ oa, double* __restrict__ ob) {
    const int k = blockIdx.x * kWG + threadIdx.x;
    if (k >= n) return;
    const int64_t o = perm[k];
    oa[k] = a[o];
    ob[k] = b[o];
}

__global__ __launch_bounds__(kWG) void fill_kernel(int n, double* __restrict__ out, double value) {
    const int k = blockIdx.x * kWG + threadIdx.x;
    if (k < n) out[k] = value;
}

// Read an 8-byte word of pinned host memory written by the host since the
// last launch: a system-scope load, so no GPU cache can answer it with an
// older copy of a reused staging slot.
__device__ __forceinline__ uint64_t host_word(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A packed work plan in pinned host memory and where it goes on the device.
struct PlanCopy {
    const uint64_t* src;
    uint64_t* dst;
    int64_t n8;        // 8-byte words
    int copy_blocks;   // leading work-groups that copy; the rest scatter
};

// Update rows in device arrays (the form of ht_set_j_particles_async).
struct DevRows {
    int n;
    const int32_t* idx;
    const double *t0, *m, *x, *v, *a, *jerk;
    int32_t lim;      // valid indices are [0, lim)
    int32_t* err;     // set when a row is dropped for its index
};

// Everything a force launch needs before it, in one launch on the compute
// queue: the work plan is pulled from pinned host memory by the first
// copy_blocks work-groups (no copy-engine transfer and no cross-engine wait),
// and the remaining work-groups write the step's update rows into records.
template <class P>
__global__ __launch_bounds__(kWG) void prep_kernel(PlanCopy pc, void* rec_base, DevRows u) {
    if (static_cast<int>(blockIdx.x) < pc.copy_blocks) {
        const int64_t stride = static_cast<int64_t>(pc.copy_blocks) * kWG;
        for (int64_t k = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; k < pc.n8; k += stride)
            pc.dst[k] = host_word(pc.src + k);
        return;
    }
    typename P::Rec* rec = static_cast<typename P::Rec*>(rec_base);
    const int b = blockIdx.x - pc.copy_blocks, nb = gridDim.x - pc.copy_blocks;
    for (int k = b * kWG + threadIdx.x; k < u.n; k += nb * kWG) {
        const int32_t j = u.idx[k];
        if (!row_index_ok(j, u.lim, u.err)) continue;
        store_rec<P>(rec, j, u.t0[k], u.m[k], u.x + 3 * k, u.v + 3 * k, u.a + 3 * k, u.jerk + 3 * k);
    }
}

// Parameters of a graph-replayed step, in a pinned host slot that the host
// rewrites before each replay (the graph's launch arguments never change).
struct GraphHdr {
    int64_t n8;           // plan words to pull
    const uint64_t* src;  // the packed plan (pinned host memory)
    int64_t n_upd;        // update rows (device arrays below)
    const int32_t* idx;
    const double *t0, *m, *x, *v, *a, *jerk;
    int64_t lim;          // valid update indices are [0, lim)
    int32_t* err;         // set when a row is dropped for its index
};
constexpr int kGraphHdrWords = 12;
static_assert(sizeof(GraphHdr) == kGraphHdrWords * 8, "GraphHdr is 12 words");

// prep_kernel for graph replays: everything it needs comes from the header.
template <class P>
__global__ __launch_bounds__(kWG) void prep_graph_kernel(const GraphHdr* hdr, uint64_t* dst, void* rec_base,
                                                         int copy_blocks) {
    __shared__ uint64_t h[kGraphHdrWords];   // the header, fetched once per work-group
    if (threadIdx.x < kGraphHdrWords)
        h[threadIdx.x] = host_word(reinterpret_cast<const uint64_t*>(hdr) + threadIdx.x);
    __syncthreads();
    if (static_cast<int>(blockIdx.x) < copy_blocks) {
        const int64_t n8 = static_cast<int64_t>(h[0]);
        const uint64_t* src = reinterpret_cast<const uint64_t*>(h[1]);
        const int64_t stride = static_cast<int64_t>(copy_blocks) * kWG;
        for (int64_t k = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; k < n8; k += stride)
            dst[k] = host_word(src + k);
        return;
    }
    const int n = static_cast<int>(h[2]);
    const int32_t* idx = reinterpret_cast<const int32_t*>(h[3]);
    const double* t0 = reinterpret_cast<const double*>(h[4]);
    const double* m = reinterpret_cast<const double*>(h[5]);
    const double* x = reinterpret_cast<const double*>(h[6]);
    const double* v = reinterpret_cast<const double*>(h[7]);
    const double* a = reinterpret_cast<const double*>(h[8]);
    const double* jerk = reinterpret_cast<const double*>(h[9]);
    const int32_t lim = static_cast<int32_t>(h[10]);
    int32_t* err = reinterpret_cast<int32_t*>(h[11]);
    typename P::Rec* rec = static_cast<typename P::Rec*>(rec_base);
    const int b = blockIdx.x - copy_blocks, nb = gridDim.x - copy_blocks;
    for (int k = b * kWG + threadIdx.x; k < n; k += nb * kWG) {
        const int32_t j = idx[k];
        if (!row_index_ok(j, lim, err)) continue;
        store_rec<P>(rec, j, t0[k], m[k], x + 3 * k, v + 3 * k, a + 3 * k, jerk + 3 * k);
    }
}

// ------------------------------------------------------------------------------------------------
// Device-resident integration: the FP64 particle state, the block scheduler
// (step 2) and the Hermite corrector with Aarseth's step (step 6) on the device.

struct DevState {
    double *x, *v, *a, *j;        // [N][3] at t0
    double *t0, *dt, *m, *pot;    // [N]
    double *acc, *jerk, *fpot;    // this step's forces, in active order
    int32_t* active;              // this step's active particles, ascending
    double* bmin;                 // per scheduler block: earliest next time
    int32_t* bcount;              // per scheduler block: particles due then
};

// What the scheduler hands the host, in pinned memory the device writes.
struct DevOut {
    double t_next;
    int64_t n_active;
    int32_t below_floor;   // a corrected step fell below 2^-40
    int32_t pad;
};

constexpr int kSchedBlocks = 1024;   // most scheduler blocks (contiguous particle ranges)

__device__ __forceinline__ double block_min(double v, double* red) {
    v = wave_ops::tree<32, 1>(v, [](double p, double q) { return fmin(p, q); });
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// One context in a scheduler launch: its state, its blocks (contiguous ranges
// of chunk particles) and where its results go.  A launch over one context
// passes its entry by value; a batched launch passes a table in device memory
// and every block finds its context by its first block.
struct SchedEntry {
    const double* t0;
    const double* dt;
    int32_t* active;
    double* bmin;
    int32_t* bcount;
    int64_t n, chunk;
    int32_t nb, first_block;
    DevOut* out;
    int32_t* active_host;     // nullptr: no host copy (device loop)
    const int32_t* halt;      // device loop: nonzero once the loop has stopped; else nullptr
};

__device__ __forceinline__ const SchedEntry& sched_entry(const SchedEntry& e0, const SchedEntry* tab, int n_tab,
                                                         int& b) {
    b = blockIdx.x;
    if (n_tab == 0) return e0;
    int lo = 0, hi = n_tab;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid].first_block <= b) lo = mid; else hi = mid;
    }
    b -= tab[lo].first_block;
    return tab[lo];
}

// pass 1: the earliest next time t0 + dt of every block's range
__global__ __launch_bounds__(kWG) void sched_min_kernel(SchedEntry e0, const SchedEntry* tab, int n_tab) {
    __shared__ double red[4];
    int b;
    const SchedEntry& e = sched_entry(e0, tab, n_tab, b);
    if (e.halt && *e.halt) return;
    const int64_t lo = b * e.chunk, hi = lo + e.chunk < e.n ? lo + e.chunk : e.n;
    double v = HUGE_VAL;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) v = fmin(v, e.t0[i] + e.dt[i]);
    v = block_min(v, red);
    if (threadIdx.x == 0) e.bmin[b] = v;
}

// pass 2: every block finds its context's t_next over all of that context's
// blocks and counts its particles due then
__global__ __launch_bounds__(kWG) void sched_count_kernel(SchedEntry e0, const SchedEntry* tab, int n_tab) {
    __shared__ double red[4];
    __shared__ int cnt[4];
    int b;
    const SchedEntry& e = sched_entry(e0, tab, n_tab, b);
    if (e.halt && *e.halt) return;
    double v = HUGE_VAL;
    for (int k = threadIdx.x; k < e.nb; k += kWG) v = fmin(v, e.bmin[k]);
    const double t_next = block_min(v, red);
    const int64_t lo = b * e.chunk, hi = lo + e.chunk < e.n ? lo + e.chunk : e.n;
    int c = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) c += e.t0[i] + e.dt[i] == t_next;
    c = wave_ops::tree<32, 1>(c, [](int p, int q) { return p + q; });
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        e.bcount[b] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        if (b == 0) e.out->t_next = t_next;
    }
}

// pass 3: every block writes its due particles, in order, after those of the
// earlier blocks of its context, into the device list and the host's copy
__global__ __launch_bounds__(kWG) void sched_write_kernel(SchedEntry e0, const SchedEntry* tab, int n_tab) {
    __shared__ double red[4];
    __shared__ int64_t part[4];
    __shared__ int wsum[4];
    int b;
    const SchedEntry& e = sched_entry(e0, tab, n_tab, b);
    if (e.halt && *e.halt) return;
    if (e.bcount[b] == 0 && b != e.nb - 1) return;   // nothing due here (the last block reports the count)
    double v = HUGE_VAL;
    for (int k = threadIdx.x; k < e.nb; k += kWG) v = fmin(v, e.bmin[k]);
    const double t_next = block_min(v, red);
    int64_t before = 0;
    for (int k = threadIdx.x; k < b; k += kWG) before += e.bcount[k];
    before = wave_ops::tree<32, 1>(before, [](int64_t p, int64_t q) { return p + q; });
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = before;
    __syncthreads();
    int64_t pos = part[0] + part[1] + part[2] + part[3];
    const int64_t lo = b * e.chunk, hi = lo + e.chunk < e.n ? lo + e.chunk : e.n;
    constexpr int kAhead = 4;   // rounds of due tests loaded together, then written in order
    for (int64_t base0 = lo; base0 < hi; base0 += kAhead * kWG) {
        bool dues[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int64_t i = base0 + u * kWG + threadIdx.x;
            dues[u] = i < hi && e.t0[i] + e.dt[i] == t_next;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int64_t base = base0 + u * kWG;
            if (base >= hi) break;
            const int64_t i = base + threadIdx.x;
            const bool due = dues[u];
            const uint64_t mask = __ballot(due);
            const int below = __popcll(mask & ((1ull << lane) - 1ull));
            __syncthreads();
            if (lane == 0) wsum[wave] = __popcll(mask);
            __syncthreads();
            int64_t at = pos + below;
            for (int w = 0; w < wave; ++w) at += wsum[w];
            if (due) {
                e.active[at] = static_cast<int32_t>(i);
                if (e.active_host) e.active_host[at] = static_cast<int32_t>(i);
            }
            pos += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        }
    }
    if (b == e.nb - 1 && threadIdx.x == 0) e.out->n_active = pos;
}

// Step 6 on the device: the Hermite corrector from (a0, jerk0) at t0 to the
// forces at t1, Aarseth's step with eta, and the block step (largest power of
// two <= min(step, dt_tree, 2 dt_old) of which t1 is a multiple); then the new
// j-record.  Same operations in the same order as the host corrector, with no
// contraction into fused multiply-adds, so both give the same bits.
__device__ __forceinline__ double dev_len3(double x, double y, double z) {
#pragma clang fp contract(off)
    return sqrt(x * x + y * y + z * z);
}

__device__ __forceinline__ double dev_quantise(double cap, double t1) {
    if (!(cap > 0.0)) return 0.0;
    int e;
    frexp(cap, &e);
    int jj = e - 1;
    if (t1 != 0.0) {
        int et;
        const double mt = frexp(fabs(t1), &et);
        const uint64_t mm = static_cast<uint64_t>(ldexp(mt, 53));
        const int v = et - 53 + __builtin_ctzll(mm);
        jj = v < jj ? v : jj;
    }
    return jj >= -40 ? ldexp(1.0, jj) : 0.0;
}

// One context in a corrector launch: its state and records, its active set
// (rows first_row .. first_row + n_active - 1 of the launch) and parameters.
// Device loop state (ht_dev_run): the step in progress and the counts so far.
struct DevLoop {
    double t_cur;        // block time of the step in progress
    int64_t n_corr;      // particles the corrector takes this step (0 once stopped)
    int64_t steps, psteps, pairs;
    int32_t halt;        // nonzero: every later kernel of the loop does nothing
    int32_t stop_after;  // the step in progress is at the stop time
    int32_t err;         // the device plan did not fit the context
    int32_t pad;
    // the call's parameters, so that the captured launches never change
    double t_stop, eta, dt_tree;
    int64_t max_steps;
};

struct CorrEntry {
    DevState s;
    void* rec;
    DevOut* out;
    int64_t n_active, first_row;
    double t1, eta, dt_tree;
    const DevLoop* loop;   // device loop: count and block time read from it; else nullptr
    // device loop: the split partials are summed here (in split order, as
    // reduce_kernel does) instead of in a launch of their own.  qmap[q] is the
    // split tile of active position q, or -1 when the force wrote q directly.
    const int32_t* qmap;
    const RTile* rtiles;
    const double* partial;
};

constexpr int kCorrBatch = 8;   // split partials loaded together by the corrector

template <class P>
__global__ __launch_bounds__(kWG) void dev_correct_kernel(CorrEntry e0, const CorrEntry* tab, int n_tab,
                                                          int64_t total, const int64_t* d_total) {
#pragma clang fp contract(off)
    // device loops: the row count is the loop's (one entry) or the batch table's (d_total)
    if (total < 0) total = d_total ? *d_total : e0.loop->n_corr;
    for (int64_t r = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; r < total;
         r += static_cast<int64_t>(gridDim.x) * kWG) {
        const CorrEntry* ep = &e0;
        if (n_tab > 0) {
            int lo = 0, hi = n_tab;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (tab[mid].first_row <= r) lo = mid; else hi = mid;
            }
            ep = tab + lo;
        }
        const CorrEntry& e = *ep;
        const DevState& s = e.s;
        typename P::Rec* rec = static_cast<typename P::Rec*>(e.rec);
        const int64_t q = r - e.first_row;
        const double t1 = e.loop ? e.loop->t_cur : e.t1;
        const int32_t i = s.active[q];
        const double D = t1 - s.t0[i];
        const double h2 = 0.5 * D, h3 = D / 3.0;
        const double D2 = D * D, D3 = D2 * D, D4 = D2 * D2, D5 = D4 * D;
        double s2[3], s3[3], s2n[3], a1[3], j1[3];
        double fp = s.fpot[q];
        const int32_t rq = e.qmap ? e.qmap[q] : -1;
        if (rq >= 0) {   // the split partials of q, summed in split order
            const RTile rt = e.rtiles[rq];
            const int64_t slot = q - rt.act_begin;
            double A[kOut];
            const double* p0 = e.partial + (rt.pbase + slot) * kOut;
            for (int u = 0; u < kOut; ++u) A[u] = p0[u];
            // kCorrBatch splits' loads in flight at once, then added in split order
            int b = 1;
            for (; b + kCorrBatch <= rt.nsplit; b += kCorrBatch) {
                double v[kCorrBatch][kOut];
                for (int w = 0; w < kCorrBatch; ++w) {
                    const double* pb = e.partial + (rt.pbase + static_cast<int64_t>(b + w) * rt.n_i + slot) * kOut;
                    for (int u = 0; u < kOut; ++u) v[w][u] = pb[u];
                }
                for (int w = 0; w < kCorrBatch; ++w)
                    for (int u = 0; u < kOut; ++u) A[u] += v[w][u];
            }
            for (; b < rt.nsplit; ++b) {
                const double* pb = e.partial + (rt.pbase + static_cast<int64_t>(b) * rt.n_i + slot) * kOut;
                for (int u = 0; u < kOut; ++u) A[u] += pb[u];
            }
            for (int d = 0; d < 3; ++d) {
                s.acc[3 * q + d] = A[d];
                s.jerk[3 * q + d] = A[3 + d];
            }
            fp = A[6];
        }
        for (int d = 0; d < 3; ++d) {
            const int64_t k = 3 * static_cast<int64_t>(i) + d;
            a1[d] = s.acc[3 * q + d];
            j1[d] = s.jerk[3 * q + d];
            const double xp = s.x[k] + D * (s.v[k] + h2 * (s.a[k] + h3 * s.j[k]));
            const double vp = s.v[k] + D * (s.a[k] + h2 * s.j[k]);
            const double diff = s.a[k] - a1[d];
            s2[d] = (-6.0 * diff - D * (4.0 * s.j[k] + 2.0 * j1[d])) / D2;
            s3[d] = (12.0 * diff + 6.0 * D * (s.j[k] + j1[d])) / D3;
            s.x[k] = xp + s2[d] * (D4 / 24.0) + s3[d] * (D5 / 120.0);
            s.v[k] = vp + s2[d] * (D3 / 6.0) + s3[d] * (D4 / 24.0);
            s.a[k] = a1[d];
            s.j[k] = j1[d];
            s2n[d] = s2[d] + D * s3[d];
        }
        const double na = dev_len3(a1[0], a1[1], a1[2]), nj = dev_len3(j1[0], j1[1], j1[2]);
        const double n2 = dev_len3(s2n[0], s2n[1], s2n[2]), n3 = dev_len3(s3[0], s3[1], s3[2]);
        const double den = nj * n3 + n2 * n2;
        const double eta = e.loop ? e.loop->eta : e.eta, dt_tree = e.loop ? e.loop->dt_tree : e.dt_tree;
        const double raw = den > 0.0 ? sqrt(eta * (na * n2 + nj * nj) / den) : dt_tree;
        double cap = dt_tree < raw ? dt_tree : raw;   // std::min(raw, dt_tree), then with 2 dt_old
        cap = 2.0 * s.dt[i] < cap ? 2.0 * s.dt[i] : cap;
        const double h = dev_quantise(cap, t1);
        if (h == 0.0) e.out->below_floor = 1;
        s.t0[i] = t1;
        s.dt[i] = h;
        s.pot[i] = fp;
        const int64_t k = 3 * static_cast<int64_t>(i);
        store_rec<P>(rec, i, t1, s.m[i], s.x + k, s.v + k, s.a + k, s.j + k);
    }
}

// ------------------------------------------------------------------------------------------------
// Device loop (ht_dev_run): block steps queued back to back with no host
// round trip.  Per step: the three scheduler passes, dev_plan_kernel (which
// first takes the step or stops the loop), the force kernel (fixed grid, counts
// read from the plan) and the corrector (count and block time read from the
// loop; it also sums the split partials, so the step needs no reduce launch).

// Take the step if its block time is at most the stop time, else stop the
// loop (and every later kernel with it).
__device__ inline void loop_gate(DevLoop* L, const DevOut* o) {
    const double t_stop = L->t_stop;
    const int64_t max_steps = L->max_steps;
    if (L->halt) {
        L->n_corr = 0;
        return;
    }
    const double t = o->t_next;
    const int64_t na = o->n_active;
    if (L->stop_after || o->below_floor || !(t <= t_stop) || L->steps >= max_steps || na < 1) {
        L->halt = 1;
        L->n_corr = 0;
        return;
    }
    L->t_cur = t;
    L->n_corr = na;
    L->steps += 1;
    L->psteps += na;
    if (t == t_stop) L->stop_after = 1;
}

// Start of a device-loop call: its parameters, counts cleared.
__global__ void loop_init_kernel(DevLoop* L, DevOut* o, double t_stop, int64_t max_steps, double eta,
                                 double dt_tree) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevLoop z{};
    z.t_stop = t_stop;
    z.max_steps = max_steps;
    z.eta = eta;
    z.dt_tree = dt_tree;
    *L = z;
    *o = DevOut{};
}

// One tile of the device plan.
struct DTile {
    int64_t jb, je;
    int32_t tb, ni;
    int32_t tl, pad;
    double cost;
};

// The group of every particle, from the group offsets (after each change of the lists).
__global__ __launch_bounds__(kWG) void group_of_kernel(int64_t n, const int64_t* __restrict__ gfirst, int32_t n_groups,
                                                       int32_t* __restrict__ pgroup) {
    const int64_t i = blockIdx.x * int64_t(kWG) + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_groups;   // gfirst[lo] <= i < gfirst[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gfirst[mid] <= i) lo = mid; else hi = mid;
    }
    pgroup[i] = lo;
}

struct PlanArgs {
    DevLoop* loop;
    const DevOut* dout;        // the scheduler's results (block time, count)
    const int32_t* active;     // this step's active particles, ascending (the scheduler's list)
    const int32_t* pgroup;     // [N] group of every particle
    const int64_t* loff;       // [groups + 1] list offsets
    int32_t* qmap;             // out: split tile of each active position or -1
    int32_t* qk;               // scratch: first active position of each active group, then n_active
    int32_t* qg;               // scratch: group of each active group
    DTile* tiles;              // scratch
    Entry* tab;                // out: the launch table (one entry)
    Item* items;               // out
    RTile* rtiles;             // out
    int64_t items_max, partial_max;
    double gather_cost, target_items;
    Desc d;                    // the context's descriptor (t, active and outputs set here)
    int8_t first_tile[257];
};

constexpr int kPlanWG = 512;

// Exclusive prefix sum over the work-group (kPlanWG threads); returns the total.
template <class V>
__device__ inline V plan_scan(V v, V* excl, V* s_wave) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const V x = wave_ops::scan_inclusive(v);
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    V before = 0, total = 0;
    for (int w = 0; w < kPlanWG / 64; ++w) {
        const V sw = s_wave[w];
        if (w < wave) before += sw;
        total += sw;
    }
    *excl = before + x - v;
    __syncthreads();
    return total;
}

// The host planner's work items (plan()), built on the device by one
// work-group: active groups, least-cost tiles, cost-based splits with the same
// quantum (the costs are whole numbers when the gather cost is, so their sum
// does not depend on the order of addition), in group order.  The order of the
// items does not change any result.
__device__ __forceinline__ void plan_body(const PlanArgs& A) {
    __shared__ int64_t s_w64[kPlanWG / 64];
    __shared__ double s_wd[kPlanWG / 64];
    __shared__ int8_t s_ft[260];   // the tile table, indexed per thread
    // up to kPlanWG active particles (the common small step): the active groups and
    // the tiles stay in LDS instead of going through memory between the phases
    __shared__ int32_t s_qk[kPlanWG + 1], s_qg[kPlanWG];
    __shared__ DTile s_tiles[kPlanWG];
    __shared__ int32_t s_g[kPlanWG];
    __shared__ int32_t s_glast;
    const int t = threadIdx.x;
    if (t < 257) s_ft[t] = A.first_tile[t];
    if (t == 0) s_glast = -1;
    DevLoop* L = A.loop;
    if (t == 0) loop_gate(L, A.dout);   // take this step or stop the loop
    __syncthreads();
    if (L->halt) {
        if (t == 0) {
            A.tab->n_items = 0;
            A.tab->n_rtiles = 0;
        }
        return;
    }
    const int64_t n = L->n_corr;
    const bool small = n <= kPlanWG;
    int32_t* QK = small ? s_qk : A.qk;
    int32_t* QG = small ? s_qg : A.qg;
    DTile* TL = small ? s_tiles : A.tiles;
    // 1-2. the group of every active particle, and the active groups (first active
    // position and group, in order); a particle's predecessor's group comes through LDS
    int64_t nq = 0;
    for (int64_t base = 0; base < n; base += kPlanWG) {
        const int64_t k = base + t;
        const int32_t g = k < n ? A.pgroup[A.active[k]] : -1;
        s_g[t] = g;
        __syncthreads();
        const int32_t gp = t > 0 ? s_g[t - 1] : s_glast;
        const int64_t f = (k < n && (k == 0 || g != gp)) ? 1 : 0;
        int64_t ex;
        const int64_t tot = plan_scan<int64_t>(f, &ex, s_w64);
        if (f) {
            QK[nq + ex] = static_cast<int32_t>(k);
            QG[nq + ex] = g;
        }
        if (t == kPlanWG - 1) s_glast = g;
        nq += tot;
    }
    if (t == 0) QK[nq] = static_cast<int32_t>(n);
    __syncthreads();
    // 3. tiles: the least-cost cover of each group's active particles
    int64_t ntile = 0;
    double total = 0.0;
    int64_t pairs = 0;
    for (int64_t base = 0; base < nq; base += kPlanWG) {
        const int64_t q = base + t;
        int64_t cnt = 0;
        if (q < nq)
            for (int64_t r = QK[q + 1] - QK[q]; r > 0;) {
                const int tl = r >= 256 ? 8 : s_ft[r];
                r -= r < (int64_t(1) << tl) ? r : (int64_t(1) << tl);
                ++cnt;
            }
        int64_t ex;
        const int64_t tot = plan_scan<int64_t>(cnt, &ex, s_w64);
        if (q < nq) {
            const int32_t g = QG[q];
            const int64_t jb = A.loff[g], je = A.loff[g + 1];
            const int64_t rounds = (je - jb + kRound - 1) / kRound;
            int64_t at = ntile + ex;
            int64_t tb = QK[q];
            for (int64_t r = QK[q + 1] - QK[q]; r > 0; ++at) {
                const int tl = r >= 256 ? 8 : s_ft[r];
                const int64_t ni = r < (int64_t(1) << tl) ? r : (int64_t(1) << tl);
                const double cost = static_cast<double>(rounds) * (A.gather_cost + static_cast<double>(1 << tl));
                TL[at] = DTile{jb, je, static_cast<int32_t>(tb), static_cast<int32_t>(ni), tl, 0, cost};
                total += cost;
                pairs += ni * (je - jb);
                tb += ni;
                r -= ni;
            }
        }
        ntile += tot;
    }
    {   // whole-number costs: the sum is exact in any order
        double ex;
        total = plan_scan<double>(total, &ex, s_wd);
        int64_t ep;
        pairs = plan_scan<int64_t>(pairs, &ep, s_w64);
    }
    __syncthreads();
    // 4. splits: the quantum doubles until the plan fits, as on the host
    double quantum = total / A.target_items;
    int attempt = 0;
    int64_t n_items = 0, n_parts = 0;
    for (;; ++attempt) {
        int64_t ci = 0, cp = 0;
        for (int64_t q = t; q < ntile; q += kPlanWG) {
            const DTile T = TL[q];
            const int64_t rsz = int64_t(kRound) * round_mult(1 << T.tl);
            const int64_t rounds = (T.je - T.jb + rsz - 1) / rsz;
            int64_t ns = (attempt > 60 || !(quantum > 0.0)) ? 1 : static_cast<int64_t>(ceil(T.cost / quantum));
            ns = ns < rounds ? ns : rounds;
            ns = ns > 1 ? ns : 1;
            if (ns == 1) {
                ci += 1;
            } else {
                const int64_t per = (rounds + ns - 1) / ns * rsz;
                const int64_t nsu = (T.je - T.jb + per - 1) / per;
                ci += nsu;
                cp += nsu * T.ni;
            }
        }
        int64_t ex;
        n_items = plan_scan<int64_t>(ci, &ex, s_w64);
        n_parts = plan_scan<int64_t>(cp, &ex, s_w64);
        if (n_items <= A.items_max && n_parts <= A.partial_max) break;
        if (attempt > 60) {   // does not fit: stop the loop before this step's force
            if (t == 0) {
                L->err = 1;
                L->halt = 1;
                L->steps -= 1;
                L->psteps -= n;
                L->n_corr = 0;
                A.tab->n_items = 0;
                A.tab->n_rtiles = 0;
            }
            return;
        }
        quantum *= 2.0;
    }
    // 5. items and split tiles, in tile order
    int64_t io = 0, po = 0, ro = 0;
    for (int64_t base = 0; base < ntile; base += kPlanWG) {
        const int64_t q = base + t;
        int64_t ci = 0, cp = 0, cr = 0, ns = 1, per = 0, nsu = 1;
        DTile T{};
        if (q < ntile) {
            T = TL[q];
            const int64_t rsz = int64_t(kRound) * round_mult(1 << T.tl);
            const int64_t rounds = (T.je - T.jb + rsz - 1) / rsz;
            ns = (attempt > 60 || !(quantum > 0.0)) ? 1 : static_cast<int64_t>(ceil(T.cost / quantum));
            ns = ns < rounds ? ns : rounds;
            ns = ns > 1 ? ns : 1;
            if (ns == 1) {
                ci = 1;
            } else {
                per = (rounds + ns - 1) / ns * rsz;
                nsu = (T.je - T.jb + per - 1) / per;
                ci = nsu;
                cp = nsu * T.ni;
                cr = 1;
            }
        }
        int64_t ei, ep, er;
        const int64_t ti = plan_scan<int64_t>(ci, &ei, s_w64);
        const int64_t tp = plan_scan<int64_t>(cp, &ep, s_w64);
        const int64_t tr = plan_scan<int64_t>(cr, &er, s_w64);
        if (q < ntile) {
            const int16_t ni = static_cast<int16_t>(T.ni), tl = static_cast<int16_t>(T.tl);
            if (ns == 1) {
                A.items[io + ei] = Item{T.jb, T.je, -1, T.tb, ni, static_cast<int16_t>(tl | kSelfTerm)};
                for (int32_t u = 0; u < T.ni; ++u) A.qmap[T.tb + u] = -1;
            } else {
                for (int32_t u = 0; u < T.ni; ++u) A.qmap[T.tb + u] = static_cast<int32_t>(ro + er);
                const int64_t pb = po + ep;
                int64_t s = 0;
                for (int64_t b = T.jb; b < T.je; b += per, ++s)
                    A.items[io + ei + s] = Item{b, b + per < T.je ? b + per : T.je, pb + s * T.ni, T.tb, ni,
                                                static_cast<int16_t>(s == 0 ? tl | kSelfTerm : tl)};
                A.rtiles[ro + er] = RTile{pb, T.tb, T.ni, static_cast<int32_t>(nsu), 0};
            }
        }
        io += ti;
        po += tp;
        ro += tr;
    }
    if (t == 0) {
        Entry& e = *A.tab;
        e.d = A.d;
        e.d.t = L->t_cur;
        e.items = A.items;
        e.rtiles = A.rtiles;
        e.first_item = 0;
        e.first_rtile = 0;
        e.n_items = io;
        e.n_rtiles = ro;
        L->pairs += pairs;
    }
}

__global__ __launch_bounds__(kPlanWG) void dev_plan_kernel(PlanArgs A) { plan_body(A); }

// ------------------------------------------------------------------------------------------------
// Batched device loop (ht_batch_dev_run): the device loop of every context of
// a batch in one chain of launches per engine step.  Each context keeps its
// own loop state, scheduler, planner scratch, plan and partials; per engine
// step the three scheduler passes run over all contexts' blocks, one planner
// work-group per context plans that context's step, a one-work-group kernel
// places the contexts' items and corrector rows one after another, and one
// force launch and one corrector launch serve them all.  A context's plan is
// the one it makes alone, so its bits are the same alone and in any batch.

// One planner work-group per context.
__global__ __launch_bounds__(kPlanWG) void dev_plan_batch_kernel(const PlanArgs* __restrict__ tab) {
    plan_body(tab[blockIdx.x]);
}

// A context's loop state and scheduler results.
struct LoopCtx {
    DevLoop* loop;
    DevOut* dout;
};

// Device words of a batched loop call.
struct LoopCounts {
    int64_t items, rtiles, rows;   // this engine step: work items, split tiles and corrector rows of all contexts
    int64_t step;                  // engine steps in which some context stepped
};

// Per-call parameters of one context (pinned host memory, read by the init kernel).
struct LoopParams {
    double t_stop, eta, dt_tree;
    int64_t max_steps;
};
static_assert(sizeof(LoopParams) == 4 * 8, "LoopParams is 4 words");

// What a call reports per context (pinned host memory, written by the results kernel).
struct LoopResult {
    int64_t steps, psteps, pairs;
    double t_cur;
    int32_t err, below_floor;
};

constexpr int kLoopTabWG = 1024;   // threads of the table kernel (one per context: kMaxBatch)
static_assert(kLoopTabWG >= kMaxBatch, "one table thread per context");

// Start of a call: every context's loop state from its parameters, counts cleared.
__global__ __launch_bounds__(kWG) void batch_loop_init_kernel(const LoopCtx* __restrict__ lc,
                                                              const LoopParams* prm, int n, LoopCounts* cnt) {
    const int k = blockIdx.x * kWG + threadIdx.x;
    if (k == 0) *cnt = LoopCounts{};
    if (k >= n) return;
    const uint64_t* w = reinterpret_cast<const uint64_t*>(prm + k);
    DevLoop z{};
    z.t_stop = __builtin_bit_cast(double, host_word(w));
    z.eta = __builtin_bit_cast(double, host_word(w + 1));
    z.dt_tree = __builtin_bit_cast(double, host_word(w + 2));
    z.max_steps = static_cast<int64_t>(host_word(w + 3));
    z.halt = z.max_steps < 1;   // a context that sits out this call: no kernel touches its state
    *lc[k].loop = z;
    *lc[k].dout = DevOut{};
}

// Exclusive prefix sum over the kLoopTabWG threads of the work-group.
__device__ inline int64_t tab_scan(int64_t v, int64_t* s_wave, int64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t x = wave_ops::scan_inclusive(v);
    __syncthreads();
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kLoopTabWG / 64; ++w) {
        if (w < wave) before += s_wave[w];
        all += s_wave[w];
    }
    *total = all;
    return before + x - v;
}

// After the planners: each context's first item, first split tile and first
// corrector row in the engine step's launches, and the step's totals; the
// time of the step (wall clock) when some context takes one.
__global__ __launch_bounds__(kLoopTabWG) void batch_loop_table_kernel(Entry* tab, CorrEntry* ctab,
                                                                      const LoopCtx* __restrict__ lc, int n,
                                                                      LoopCounts* cnt, int64_t* ts, int64_t ts_max) {
    __shared__ int64_t s_wave[kLoopTabWG / 64];
    const int k = threadIdx.x;
    const bool on = k < n;
    int64_t ti, tr, tc;
    const int64_t ei = tab_scan(on ? tab[k].n_items : 0, s_wave, &ti);
    const int64_t er = tab_scan(on ? tab[k].n_rtiles : 0, s_wave, &tr);
    const int64_t ec = tab_scan(on ? lc[k].loop->n_corr : 0, s_wave, &tc);
    if (on) {
        tab[k].first_item = ei;
        tab[k].first_rtile = er;
        ctab[k].first_row = ec;
    }
    if (k == 0) {
        cnt->items = ti;
        cnt->rtiles = tr;
        cnt->rows = tc;
        if (tc > 0) {
            const int64_t st = cnt->step;
            if (st < ts_max) ts[st] = static_cast<int64_t>(wall_clock64());
            cnt->step = st + 1;
        }
    }
}

// End of a call: every context's counts and state, and the step times, into pinned memory.
__global__ __launch_bounds__(kWG) void batch_loop_results_kernel(const LoopCtx* __restrict__ lc, int n,
                                                                 LoopResult* out, const LoopCounts* cnt,
                                                                 const int64_t* ts, int64_t ts_max, int64_t* ts_out) {
    const int k = blockIdx.x * kWG + threadIdx.x;
    if (k < n) {
        const DevLoop& L = *lc[k].loop;
        out[k] = LoopResult{L.steps, L.psteps, L.pairs, L.t_cur, L.err, lc[k].dout->below_floor};
    }
    const int64_t m = cnt->step < ts_max ? cnt->step : ts_max;
    for (int64_t q = k; q < m; q += static_cast<int64_t>(gridDim.x) * kWG) ts_out[1 + q] = ts[q];
    if (k == 0) {
        ts_out[0] = m;
        ts_out[1 + m] = static_cast<int64_t>(wall_clock64());
    }
}

// Batched j-memory update: rows of several clusters in one launch.
struct UpdEntry {
    void* rec;            // the cluster's records
    int64_t first_row;    // its first row in the launch
    const ht_row* rows;   // its rows (pinned host memory)
    int64_t lim;          // its particle count: valid row indices are [0, lim)
};

__device__ __forceinline__ int find_upd(const UpdEntry* tab, int n_tab, int64_t r) {
    int lo = 0, hi = n_tab;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid].first_row <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// The launch table and the rows are read straight from pinned host memory
// (system-scope loads, see host_word), so an update costs one launch and no
// device copy; every work-group keeps the table in LDS.
template <class P>
__global__ __launch_bounds__(kWG) void scatter_rows_kernel(const UpdEntry* __restrict__ tab, int n_tab, int64_t total,
                                                           int32_t* err) {
    static_assert(sizeof(ht_row) == 15 * 8, "ht_row is 15 words");
    static_assert(sizeof(UpdEntry) == 32, "UpdEntry is 4 words");
    __shared__ UpdEntry stab[kMaxBatch];
    for (int q = threadIdx.x; q < 4 * n_tab; q += kWG)
        reinterpret_cast<uint64_t*>(stab)[q] = host_word(reinterpret_cast<const uint64_t*>(tab) + q);
    __syncthreads();
    for (int64_t r = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; r < total;
         r += static_cast<int64_t>(gridDim.x) * kWG) {
        const int k = find_upd(stab, n_tab, r);
        const uint64_t* w = reinterpret_cast<const uint64_t*>(stab[k].rows + (r - stab[k].first_row));
        uint64_t raw[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) raw[q] = host_word(w + q);
        double f[14];
#pragma unroll
        for (int q = 0; q < 14; ++q) f[q] = __builtin_bit_cast(double, raw[q + 1]);
        const int32_t idx = static_cast<int32_t>(static_cast<uint32_t>(raw[0]));
        if (!row_index_ok(idx, static_cast<int32_t>(stab[k].lim), err)) continue;
        // f: t0, m, x[3], v[3], a[3], jerk[3]
        store_rec<P>(static_cast<typename P::Rec*>(stab[k].rec), idx, f[0], f[1], f + 2, f + 5, f + 8, f + 11);
    }
}

// ------------------------------------------------------------------------------------------------
// host side
size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

int ceil_log2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

constexpr double kGatherCostDefault = 12.0;    // work-plan cost of one round's gather, in pairs per lane (measured best 8-16)
constexpr double kTargetItemsDefault = 2048.0; // work items a call is split towards (2 per resident slot)
constexpr int kStageRows = 1 << 16;  // rows per host->device upload chunk
constexpr int kMaxBins = 16;         // runs of a placed plan (one per XCD)

struct Layout {
    size_t jcap, stored, vel;
    size_t off_rec, off_prec;
    size_t off_entries, off_plan, off_partial, off_out, off_stage;
    int64_t items_max, partial_max;
    size_t plan_bytes;  // launch table + items + reduce tiles + active ids, packed per call
    size_t total;
};

bool layout_of(const ht_config& c, Layout& L) {
    if (c.n_max < 1 || c.node_max < 0 || c.group_max < 1 || c.list_max < 1 || c.active_max < 1) return false;
    if (c.precision != HT_PREC_FP64 && c.precision != HT_PREC_MIXED) return false;
    if (c.predict_mode != HT_PREDICT_FUSED && c.predict_mode != HT_PREDICT_EAGER) return false;
    if (static_cast<int64_t>(c.n_max) + c.node_max > INT32_MAX - 1) return false;
    L.jcap = static_cast<size_t>(c.n_max) + static_cast<size_t>(c.node_max);
    L.stored = c.precision == HT_PREC_FP64 ? sizeof(double) : sizeof(float);
    L.vel = L.stored;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.off_rec = take(L.jcap * 128);
    const bool eager = c.predict_mode == HT_PREDICT_EAGER;
    L.off_prec = take(eager ? L.jcap * 64 : 0);
    L.off_entries = take(static_cast<size_t>(c.list_max) * 4);
    L.items_max = 4 * (static_cast<int64_t>(c.group_max) + c.active_max / 256 + 1) + 4096;
    L.partial_max = 2 * static_cast<int64_t>(c.active_max) + 65536;
    L.plan_bytes = align_up(kMaxBatch * sizeof(Entry)) + align_up(static_cast<size_t>(L.items_max) * sizeof(Item)) +
                   align_up(static_cast<size_t>(L.items_max) * sizeof(RTile)) +
                   align_up(static_cast<size_t>(c.active_max) * 4) +
                   align_up(static_cast<size_t>(L.items_max) * 8) +   // item run cursors (run-length lists)
                   align_up(static_cast<size_t>(c.active_max)) +      // member indices (union tiles)
                   align_up((kMaxBins + 1) * 8) + 256;                 // run offsets of a placed plan
    L.off_plan = take(L.plan_bytes);
    L.off_partial = take(static_cast<size_t>(L.partial_max) * kOut * 8);
    L.off_out = take(static_cast<size_t>(c.active_max) * kOut * 8);
    L.off_stage = take(static_cast<size_t>(kStageRows) * (4 + 8 + 8 + 4 * 24));
    L.total = o;
    return true;
}

// Optional timing of force-kernel launches: HIP events around each launch.
struct Timing {
    bool enabled = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int64_t pairs = 0;
};

// A ring of pinned host slots, each mirroring a device region byte for byte,
// so the host can pack several calls ahead of the device.  A slot is reused
// once the copy that read it has completed.
struct PinnedRing {
    static constexpr int kSlots = 4;
    char* base = nullptr;
    size_t slot_bytes = 0;
    hipEvent_t ev[kSlots] = {};
    bool pending[kSlots] = {};
    int slot = 0;
    char* host() const { return base + static_cast<size_t>(slot) * slot_bytes; }
};

}  // namespace

struct ht_ctx {
    ht_config cfg{};
    Layout L{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;
    bool own_ws = false;
    // Host pinned staging: a ring of plan slots (each mirrors the device plan
    // region byte for byte) so the host can plan several calls ahead of the
    // device, then room for results read back to host arrays.  A slot is
    // reused once the copy that read it has completed.
    static constexpr int kPlanSlots = 4;
    char* h_pinned = nullptr;
    char* h_out = nullptr;
    int32_t* h_err = nullptr;   // set by a kernel that dropped an update row for its index
    hipEvent_t slot_free[kPlanSlots] = {};
    bool slot_pending[kPlanSlots] = {};
    int slot = 0;
    // j-memory state
    int32_t n = 0, n_nodes = 0, n_groups = 0;
    int64_t n_entries = 0;
    bool have_particles = false, have_nodes = false, have_lists = false, predicted = false;
    double t_pred = 0.0;
    std::vector<int64_t> group_first, list_off;
    // last call statistics
    int64_t last_pairs = 0;
    int32_t last_items = 0;
    Timing tm;
    // per-call scratch: marks for repeated update indices (generation-stamped)
    std::vector<uint32_t> mark;
    uint32_t mark_gen = 0;
    // work-plan tuning (see plan())
    double gather_cost = kGatherCostDefault;
    double target_items = kTargetItemsDefault;
    int8_t first_tile[257] = {};   // least-cost tiling for the gather cost (tile_table)
    // placement over XCDs (ht_set_placement): placement runs requested (1: off),
    // the device's XCD count, and the last plan's run offsets and longest run
    int32_t placement = 1, n_xcc = 1;
    int32_t n_bins = 1;
    int64_t bin_off[kMaxBins + 1] = {};
    int64_t bin_max = 0;
    std::vector<uint8_t> item_bin, sort_bins;
    // ht_step_graph: captured step graphs, one per pinned header slot, so the
    // host can fill headers while earlier replays are still running
    hipStream_t cap_stream = nullptr;
    static constexpr int kGraphSlots = 4;
    hipGraph_t graph[kGraphSlots] = {};
    hipGraphExec_t gexec[kGraphSlots] = {};
    hipEvent_t hdr_free[kGraphSlots] = {};
    bool hdr_pending[kGraphSlots] = {};
    int gslot = 0;
    GraphHdr* h_hdr = nullptr;
    // device-resident integration (ht_state_enable): FP64 state and scheduler
    // buffers on the device, the scheduler's results in pinned host memory
    DevState ds{};
    char* ds_mem = nullptr;
    bool own_ds = false;   // ds_mem allocated by the library (ht_state_enable), not the caller's
    // device loop (ht_dev_run): its state, the scheduler's results in device
    // memory, the group and list offsets and the planner's scratch
    DevLoop* d_loop = nullptr;
    DevOut* d_dout = nullptr;
    int64_t* d_gfirst = nullptr;
    int64_t* d_loff = nullptr;
    int32_t *d_gk = nullptr, *d_qk = nullptr, *d_qg = nullptr, *d_pgroup = nullptr;
    DTile* d_tiles = nullptr;
    hipGraph_t loop_graph = nullptr;      // kLoopGraphSteps device-loop steps, captured once
    hipGraphExec_t loop_exec = nullptr;
    double loop_tuning[2] = {-1.0, -1.0}; // the tuning the graph's planner launches carry
    int32_t loop_self_once = -1;          // and the descriptor's self_once
    // every list holds each particle of its group exactly once (checked when
    // host lists are set; true for the device builder's lists by construction)
    bool self_once_lists = false;
    DevOut* h_dout = nullptr;
    int32_t* h_active = nullptr;
    double dev_t_next = 0.0;
    int64_t dev_n_active = -1;   // active set of the last ht_dev_next_block, -1 once stepped
    // run-length lists (HT_LISTS_RUNS, set by ht_set_list_form): runs of
    // consecutive combined indices over each list, the groups' node copies
    // (indices copy_base.. in their own records), and the host's copy of the
    // run positions for the planner's per-item run cursors
    int32_t list_form = HT_LISTS_CSR;
    int32_t* d_run_start = nullptr;
    int64_t* d_run_pos = nullptr;
    char* d_copy_rec = nullptr;
    int32_t* d_copy_src = nullptr;
    size_t run_cap = 0, copy_cap = 0;
    int64_t n_runs = 0, n_copies = 0;
    std::vector<int64_t> run_pos;
    std::vector<int64_t> item_runs;
    // union tiles (HT_LISTS_UNION, ht_set_union_width): runs of union_width
    // consecutive groups, their union lists (entries and member masks on the
    // device, offsets and lengths on the host) and the per-call member index
    // of each active position
    int32_t union_width = 4;
    int32_t* d_uent = nullptr;
    uint8_t* d_umask = nullptr;
    size_t ucap = 0;
    std::vector<int64_t> u_off;
    std::vector<uint8_t> act_member;
    int64_t union_items = 0;   // union-tile items in the last plan
    // scratch for planning
    std::vector<Item> items;
    std::vector<RTile> rtiles;
    std::vector<Item> sort_items;
    std::vector<uint32_t> sort_keys, sort_count;

    template <class T>
    T* dev(size_t off) const { return reinterpret_cast<T*>(ws + off); }

    Desc desc() const {
        Desc d{};
        d.rec = ws + L.off_rec;
        d.prec = ws + L.off_prec;
        d.entries = dev<int32_t>(L.off_entries);
        d.partial = dev<double>(L.off_partial);
        d.t = t_pred;
        d.eps2 = cfg.eps2;
        d.self_once = self_once_lists && cfg.eps2 > 0.0 ? 1 : 0;
        if (list_form == HT_LISTS_UNION) {
            d.u_entries = d_uent;
            d.u_mask = d_umask;
        }
        if (list_form == HT_LISTS_RUNS) {
            d.run_start = d_run_start;
            d.run_pos = d_run_pos;
            d.copy_rec = d_copy_rec;
            d.n_runs = n_runs;
            d.copy_base = n + n_nodes;
        }
        return d;
    }

    char* plan_host() const { return h_pinned + static_cast<size_t>(slot) * L.plan_bytes; }
    // Wait until the current plan slot may be overwritten.
    int slot_acquire() {
        if (slot_pending[slot]) {
            HT_HIP(hipEventSynchronize(slot_free[slot]));
            slot_pending[slot] = false;
        }
        return HT_OK;
    }
    // The copy reading the current slot is queued: mark it and move on.
    int slot_release() {
        HT_HIP(hipEventRecord(slot_free[slot], stream));
        slot_pending[slot] = true;
        slot = (slot + 1) % kPlanSlots;
        return HT_OK;
    }
    // After a stream synchronisation every slot is free.
    void slots_all_free() {
        for (int k = 0; k < kPlanSlots; ++k) slot_pending[k] = false;
    }
};

// Batched engine object: its own plan and update regions, big enough for all
// clusters of one engine step, so a step costs one update copy + one scatter
// and one plan copy + one force launch (+ one reduce) for every cluster.
struct ht_batch {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    int32_t max_clusters = 0;
    int64_t max_items = 0, max_active = 0, max_rows = 0;
    size_t plan_bytes = 0, rows_bytes = 0;
    char* ws = nullptr;
    bool own_ws = false;
    PinnedRing plan_ring, rows_ring;
    Timing tm;
    int64_t last_pairs = 0;
    int32_t last_items = 0;
    std::vector<Entry> tab;
    std::vector<UpdEntry> utab;
    int32_t* h_err = nullptr;   // set by the row scatter when it dropped a row for its index
    // batched device loop (ht_batch_dev_run): its tables sit in the workspace
    // after the plan region; the graph of kLoopGraphSteps engine steps is
    // captured for one set of contexts (and their sizes and tunings) and kept
    // until the set changes
    char* loop_ws = nullptr;
    std::vector<ht_ctx*> loop_ctxs;
    std::vector<double> loop_key;
    int32_t loop_blocks = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t loop_graph = nullptr;
    hipGraphExec_t loop_exec = nullptr;
    LoopParams* h_lparams = nullptr;   // pinned: per-call parameters
    LoopResult* h_lres = nullptr;      // pinned: per-call results
    int64_t* h_ts = nullptr;           // pinned: engine-step times of the last call
};

namespace {

int grid_for(int64_t items) {
    return static_cast<int>(std::min<int64_t>(std::max<int64_t>(items, 1), 1 << 20));
}

bool check_vectors(const double* const* ptrs, int count) {
    for (int k = 0; k < count; ++k)
        if (!ptrs[k]) return false;
    return true;
}

// Work plan of one force call.  The active particles of one group (ids are
// strictly increasing, groups are contiguous ranges) form i-tiles of T = 1,
// 2, 4, ..., 256 slots.  A tile's cost is modelled as
//   rounds * (gather_cost + T),  rounds = ceil(list length / 256),
// i.e. per round of 256 entries one gather-and-predict (worth about
// gather_cost pairs of arithmetic per lane) plus T pairs per lane, idle slots
// included.  A group's n active particles are covered by the tiles of least
// total cost: 140 becomes 128 + 16 (cost 2 gc + 144) rather than one part-
// filled 256 (gc + 256), while 3 stays one tile of 4.  Tiles are
// only split (into list ranges whose partials are summed afterwards) when the
// call has too little work to fill the chip: each tile gets about
// cost / (total / target_items) items.  Items are then ordered by decreasing
// cost: the hardware hands work-groups out in index order as slots free up,
// which makes that a longest-first schedule.  The plan depends only on this
// context's lists, active set and tuning, so a context gives the same bits
// alone and in a batched launch.

struct Tile {
    int64_t jb, je;
    int32_t tb, ni;
    int tl;
    double cost;
    bool uni;   // over a union list (union tiles)
};

// first_tile[r] (r = 1..256): log2 of the first tile in the least-cost cover
// of r active particles by power-of-two tiles, the cost of a tile being
// gather_cost + T.  Either one tile of the next power of two holds all r, or
// a full tile of the largest power of two below r is followed by the best
// cover of the rest.
void tile_table(double gather_cost, int8_t* first_tile) {
    double best[257];
    best[0] = 0.0;
    for (int r = 1; r <= 256; ++r) {
        const int up = ceil_log2(r);
        double b = gather_cost + static_cast<double>(1 << up);
        int8_t f = static_cast<int8_t>(up);
        const int down = (1 << up) == r ? up : up - 1;
        if ((1 << down) < r) {
            const double alt = gather_cost + static_cast<double>(1 << down) + best[r - (1 << down)];
            if (alt < b) {
                b = alt;
                f = static_cast<int8_t>(down);
            }
        }
        best[r] = b;
        first_tile[r] = f;
    }
}

int plan(ht_ctx* c, int32_t n_active, const int32_t* ids, bool direct, bool place = false) {
    auto& items = c->items;
    auto& rtiles = c->rtiles;
    static thread_local std::vector<Tile> tiles;
    tiles.clear();
    int64_t pairs = 0;
    double total = 0.0;
    // the tiles of least modelled cost over a list of len entries for the
    // active positions [tb, e), and what they cost
    auto cover_cost = [c](int32_t n, int64_t len) {
        const double rounds = static_cast<double>((len + kRound - 1) / kRound);
        double cost = 0.0;
        for (int32_t r = n; r > 0;) {
            const int tl = r >= 256 ? 8 : c->first_tile[r];
            cost += rounds * (c->gather_cost + static_cast<double>(1 << tl));
            r -= std::min<int32_t>(r, 1 << tl);
        }
        return cost;
    };
    auto cover = [&](int64_t jb, int64_t je, int32_t tb, int32_t e, bool uni) {
        while (tb < e) {
            const int32_t r = e - tb;
            const int tl = r >= 256 ? 8 : c->first_tile[r];
            const int32_t ni = std::min<int32_t>(r, 1 << tl);
            const int64_t rounds = (je - jb + kRound - 1) / kRound;
            const double cost = static_cast<double>(rounds) * (c->gather_cost + static_cast<double>(1 << tl));
            tiles.push_back(Tile{jb, je, tb, ni, tl, cost, uni});
            total += cost;
            tb += ni;
        }
    };
    const bool uni = c->list_form == HT_LISTS_UNION && !direct;
    if (uni) c->act_member.assign(static_cast<size_t>(n_active), 0);
    size_t g = 0;
    int32_t k = 0;
    while (k < n_active) {
        if (direct) {
            cover(0, c->n, k, n_active, false);
            pairs += static_cast<int64_t>(n_active) * c->n;
            break;
        }
        while (c->group_first[g + 1] <= ids[k]) ++g;
        if (!uni) {
            const int64_t ge = c->group_first[g + 1];
            int32_t e = k;
            while (e < n_active && ids[e] < ge) ++e;
            cover(c->list_off[g], c->list_off[g + 1], k, e, false);
            pairs += static_cast<int64_t>(e - k) * (c->list_off[g + 1] - c->list_off[g]);
            k = e;
            continue;
        }
        // union tiles: the run of groups holding group g, its members' active
        // ranges, and the cheaper of per-group tiles and tiles over the union
        const int32_t w = c->union_width;
        const int32_t run = static_cast<int32_t>(g) / w;
        const int32_t g0 = run * w, g1 = std::min<int32_t>(c->n_groups, g0 + w);
        int32_t starts[9];
        int32_t e = k;
        double sep = 0.0;
        int64_t run_pairs = 0;
        for (int32_t q = g0; q < g1; ++q) {
            starts[q - g0] = e;
            const int64_t ge = c->group_first[q + 1];
            const int32_t b0 = e;
            while (e < n_active && ids[e] < ge) ++e;
            const int64_t len = c->list_off[q + 1] - c->list_off[q];
            if (e > b0) sep += cover_cost(e - b0, len);
            run_pairs += static_cast<int64_t>(e - b0) * len;
        }
        starts[g1 - g0] = e;
        const int64_t ub = c->u_off[run], ue = c->u_off[run + 1];
        if (cover_cost(e - k, ue - ub) < sep) {
            for (int32_t q = g0; q < g1; ++q)
                for (int32_t a = starts[q - g0]; a < starts[q - g0 + 1]; ++a)
                    c->act_member[a] = static_cast<uint8_t>(q - g0);
            cover(ub, ue, k, e, true);
        } else {
            for (int32_t q = g0; q < g1; ++q)
                if (starts[q - g0 + 1] > starts[q - g0])
                    cover(c->list_off[q], c->list_off[q + 1], starts[q - g0], starts[q - g0 + 1], false);
        }
        pairs += run_pairs;
        g = static_cast<size_t>(g1 - 1);
        k = e;
    }
    double quantum = total / c->target_items;
    for (int attempt = 0;; ++attempt) {
        items.clear();
        rtiles.clear();
        int64_t pslots = 0;
        for (const Tile& t : tiles) {
            const int64_t rsz = static_cast<int64_t>(kRound) * round_mult(1 << t.tl);   // the kernel's round
            const int64_t rounds = (t.je - t.jb + rsz - 1) / rsz;
            int64_t ns = attempt > 60 ? 1 : static_cast<int64_t>(std::ceil(t.cost / quantum));
            ns = std::max<int64_t>(1, std::min<int64_t>(ns, rounds));
            if (ns == 1) {
                items.push_back(Item{t.jb, t.je, -1, t.tb, static_cast<int16_t>(t.ni),
                                     static_cast<int16_t>(t.tl | kSelfTerm | (t.uni ? kUnion : 0))});
                continue;
            }
            const int64_t per = (rounds + ns - 1) / ns * rsz;   // entries per split, whole rounds
            int32_t nsu = 0;
            for (int64_t b = t.jb; b < t.je; b += per, ++nsu)
                items.push_back(Item{b, std::min(t.je, b + per), pslots + static_cast<int64_t>(nsu) * t.ni, t.tb,
                                     static_cast<int16_t>(t.ni),
                                     static_cast<int16_t>((nsu == 0 ? t.tl | kSelfTerm : t.tl) |
                                                          (t.uni ? kUnion : 0))});
            rtiles.push_back(RTile{pslots, t.tb, t.ni, nsu, 0});
            pslots += static_cast<int64_t>(nsu) * t.ni;
        }
        if (static_cast<int64_t>(items.size()) <= c->L.items_max && pslots <= c->L.partial_max) break;
        if (attempt > 60) return fail(HT_ERANGE, "work plan exceeds the context's item capacity");
        quantum *= 2.0;
    }
    // Placement (more than one run requested, list items): the items, still in
    // group order, i.e. in space-filling order of their groups, are cut into
    // n_bins runs of equal modelled cost, an item going to the run that holds
    // the middle of its cost.  Neighbouring groups' lists share most of their
    // nodes and many particles, so a run's items reuse each other's records in
    // the L2 of the XCD that runs them; a long list's splits still spread over
    // the runs.
    const double gc = c->gather_cost;
    auto item_cost = [gc](const Item& it) {
        return static_cast<double>((it.j_end - it.j_begin + kRound - 1) / kRound) *
               (gc + static_cast<double>(1 << (it.tile_log2 & kTileMask)));
    };
    const int nb = (place && c->placement > 1 && !direct && items.size() > 1) ? c->placement : 1;
    auto& ib = c->item_bin;
    ib.assign(items.size(), 0);
    if (nb > 1) {
        double tot = 0.0, cum = 0.0;
        for (const Item& it : items) tot += item_cost(it);
        for (size_t q = 0; q < items.size(); ++q) {
            const double w = item_cost(items[q]);
            const int b = static_cast<int>(static_cast<double>(nb) * (cum + 0.5 * w) / tot);
            ib[q] = static_cast<uint8_t>(std::min(std::max(b, 0), nb - 1));
            cum += w;
        }
    }
    // Longest first, to 1/8 of an octave: a counting sort on the sign,
    // exponent and top three mantissa bits of the modelled cost (monotone in
    // the cost for positive doubles), equal keys in plan order, so the order
    // is deterministic and linear in the number of items.  A placed plan is
    // then ordered by run, stably, so each run is longest first.
    auto& keys = c->sort_keys;
    keys.resize(items.size());
    uint32_t kmin = UINT32_MAX, kmax = 0;
    for (size_t q = 0; q < items.size(); ++q) {
        const double cost = item_cost(items[q]);
        uint64_t bits;
        std::memcpy(&bits, &cost, 8);
        keys[q] = static_cast<uint32_t>(bits >> 49);
        kmin = std::min(kmin, keys[q]);
        kmax = std::max(kmax, keys[q]);
    }
    auto& out = c->sort_items;
    auto& ob = c->sort_bins;
    if (items.size() > 1 && kmax > kmin) {
        auto& count = c->sort_count;
        count.assign(static_cast<size_t>(kmax - kmin) + 2, 0);
        for (uint32_t k : keys) ++count[kmax - k + 1];   // bucket 0 = largest cost
        for (size_t b = 1; b < count.size(); ++b) count[b] += count[b - 1];
        out.resize(items.size());
        ob.resize(items.size());
        for (size_t q = 0; q < items.size(); ++q) {
            const uint32_t at = count[kmax - keys[q]]++;
            out[at] = items[q];
            ob[at] = ib[q];
        }
        items.swap(out);
        ib.swap(ob);
    }
    c->n_bins = nb;
    if (nb > 1) {
        int64_t* off = c->bin_off;
        std::fill(off, off + nb + 1, 0);
        for (uint8_t b : ib) ++off[b + 1];
        c->bin_max = 0;
        for (int b = 0; b < nb; ++b) {
            c->bin_max = std::max(c->bin_max, off[b + 1]);
            off[b + 1] += off[b];
        }
        int64_t at[kMaxBins];
        std::copy(off, off + nb, at);
        out.resize(items.size());
        for (size_t q = 0; q < items.size(); ++q) out[at[ib[q]]++] = items[q];
        items.swap(out);
    }
    c->item_runs.clear();
    if (c->list_form == HT_LISTS_RUNS && !direct) {   // the run holding each item's first position
        auto& ir = c->item_runs;
        ir.resize(items.size());
        for (size_t q = 0; q < items.size(); ++q)
            ir[q] = static_cast<int64_t>(std::upper_bound(c->run_pos.begin(), c->run_pos.end(), items[q].j_begin) -
                                         c->run_pos.begin()) - 1;
    }
    c->union_items = 0;
    if (uni)
        for (const Item& it : items) c->union_items += (it.tile_log2 & kUnion) ? 1 : 0;
    c->last_pairs = pairs;
    c->last_items = static_cast<int32_t>(items.size());
    return HT_OK;
}

int validate_active(const ht_ctx* c, int32_t n_active, const int32_t* ids) {
    if (n_active < 0) return fail(HT_EINVAL, "n_active < 0");
    if (n_active > c->cfg.active_max) return fail(HT_ERANGE, "n_active %d over capacity %d", n_active, c->cfg.active_max);
    if (n_active > 0 && !ids) return fail(HT_EINVAL, "active_ids is NULL");
    for (int32_t k = 0; k < n_active; ++k) {
        if (ids[k] < 0 || ids[k] >= c->n) return fail(HT_EINVAL, "active id %d outside [0, %d)", ids[k], c->n);
        if (k > 0 && ids[k] <= ids[k - 1]) return fail(HT_EINVAL, "active ids not strictly increasing at %d", k);
    }
    return HT_OK;
}

// Pack one context's items, reduce tiles and active ids into its pinned
// staging from byte offset `at` on (the device plan region mirrors that
// staging byte for byte); point the launch entry at the device copies.
// Returns the end of the packed bytes.
size_t pack_plan_into(ht_ctx* c, char* hs, char* dv, size_t at, int32_t n_active, const int32_t* ids, double* acc,
                      double* jerk, double* pot, Entry& e) {
    const size_t o_items = align_up(at);
    const size_t b_items = c->items.size() * sizeof(Item);
    const size_t o_rt = align_up(o_items + b_items);
    const size_t b_rt = c->rtiles.size() * sizeof(RTile);
    const size_t o_act = align_up(o_rt + b_rt);
    std::memcpy(hs + o_items, c->items.data(), b_items);
    if (b_rt) std::memcpy(hs + o_rt, c->rtiles.data(), b_rt);
    std::memcpy(hs + o_act, ids, static_cast<size_t>(n_active) * 4);
    e.d = c->desc();
    size_t end = o_act + static_cast<size_t>(n_active) * 4;
    if (c->list_form == HT_LISTS_RUNS) {   // each item's first run, in item order
        const size_t o_ir = align_up(end);
        std::memcpy(hs + o_ir, c->item_runs.data(), c->item_runs.size() * 8);
        e.d.item_runs = reinterpret_cast<const int64_t*>(dv + o_ir);
        end = o_ir + c->item_runs.size() * 8;
    }
    if (c->list_form == HT_LISTS_UNION && c->act_member.size() == static_cast<size_t>(n_active)) {
        const size_t o_am = align_up(end);   // each active position's member index in its run
        std::memcpy(hs + o_am, c->act_member.data(), static_cast<size_t>(n_active));
        e.d.act_member = reinterpret_cast<const uint8_t*>(dv + o_am);
        end = o_am + static_cast<size_t>(n_active);
    }
    e.d.active = reinterpret_cast<const int32_t*>(dv + o_act);
    e.d.acc = acc;
    e.d.jerk = jerk;
    e.d.pot = pot;
    e.items = reinterpret_cast<const Item*>(dv + o_items);
    e.rtiles = reinterpret_cast<const RTile*>(dv + o_rt);
    return end;
}

size_t pack_plan(ht_ctx* c, size_t at, int32_t n_active, const int32_t* ids, double* acc, double* jerk, double* pot,
                 Entry& e) {
    return pack_plan_into(c, c->plan_host(), c->ws + c->L.off_plan, at, n_active, ids, acc, jerk, pot, e);
}

// Pull `bytes` of a packed plan from pinned host memory into the device plan
// region and write update rows `u`, in one prep_kernel launch.
template <class P>
int launch_prep(hipStream_t stream, const char* h_src, char* d_dst, size_t bytes, void* rec, const DevRows& u) {
    PlanCopy pc{reinterpret_cast<const uint64_t*>(h_src), reinterpret_cast<uint64_t*>(d_dst),
                static_cast<int64_t>((bytes + 7) / 8), 0};
    pc.copy_blocks = static_cast<int>(std::min<int64_t>((pc.n8 + kWG - 1) / kWG, 2048));
    const int scatter_blocks = u.n > 0 ? std::min((u.n + kWG - 1) / kWG, 65536) : 0;
    if (pc.copy_blocks + scatter_blocks == 0) return HT_OK;
    prep_kernel<P><<<pc.copy_blocks + scatter_blocks, kWG, 0, stream>>>(pc, rec, u);
    HT_HIP(hipGetLastError());
    return HT_OK;
}

int launch_prep_any(int precision, hipStream_t stream, const char* h_src, char* d_dst, size_t bytes, void* rec,
                    const DevRows& u) {
    if (precision == HT_PREC_FP64) return launch_prep<PrecFp64>(stream, h_src, d_dst, bytes, rec, u);
    return launch_prep<PrecMixed>(stream, h_src, d_dst, bytes, rec, u);
}

// One host-to-device copy of the packed prefix [0, end) of the plan.
int copy_plan(ht_ctx* c, size_t end) {
    HT_HIP(hipMemcpyAsync(c->ws + c->L.off_plan, c->plan_host(), end, hipMemcpyHostToDevice, c->stream));
    // the slot is free once this copy is done, not the kernels
    return c->slot_release();
}

template <class P>
int launch_force(hipStream_t stream, bool eager, Timing& tm, const Entry* d_tab, int n_tab, int64_t n_items,
                 int64_t n_rtiles, bool direct, int64_t pairs, bool runs = false, const int64_t* d_bins = nullptr,
                 int n_bins = 1, int64_t bin_max = 0, bool uni = false) {
    const int grid = d_bins ? static_cast<int>(n_bins * bin_max) : grid_for(n_items);
    using Kern = void (*)(const Entry*, int, int64_t, const int64_t*, const int64_t*, int);
    Kern kern;
    if (direct) kern = eager ? force_kernel<P, true, true> : force_kernel<P, false, true>;
    else if (runs) kern = force_kernel<P, false, false, true>;
    else if (uni) kern = force_kernel<P, false, false, false, true>;
    else kern = eager ? force_kernel<P, true, false> : force_kernel<P, false, false>;
    const int64_t* counts = nullptr;
    if (tm.enabled) {
        // Timing: the extended launch stamps the two events with the kernel's
        // own start and end, so the time excludes the dispatch around it.
        while (tm.pool.size() < tm.used + 2) {
            hipEvent_t e;
            HT_HIP(hipEventCreate(&e));
            tm.pool.push_back(e);
        }
        hipEvent_t ev_a = tm.pool[tm.used], ev_b = tm.pool[tm.used + 1];
        tm.used += 2;
        tm.pairs += pairs;
        void* args[] = {&d_tab, &n_tab, &n_items, &counts, &d_bins, &n_bins};
        HT_HIP(hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kWG), args, 0, stream, ev_a,
                                  ev_b, 0));
    } else {
        kern<<<grid, kWG, 0, stream>>>(d_tab, n_tab, n_items, counts, d_bins, n_bins);
        HT_HIP(hipGetLastError());
    }
    if (n_rtiles > 0) {
        reduce_kernel<<<grid_for(n_rtiles), kWG, 0, stream>>>(d_tab, n_tab, n_rtiles);
        HT_HIP(hipGetLastError());
    }
    return HT_OK;
}

// A kernel dropped an update row whose particle index (read from device or
// pinned memory) was outside [0, N): report it once, at the first
// synchronisation that follows.
int take_row_error(int32_t* w) {
    if (w && __atomic_load_n(w, __ATOMIC_ACQUIRE) != 0) {
        __atomic_store_n(w, 0, __ATOMIC_RELEASE);
        return fail(HT_ERANGE, "an update row named a particle index outside [0, N); the row was dropped");
    }
    return HT_OK;
}

// Wait for the context's stream; every plan slot is free afterwards.  Returns
// HT_ERANGE when a kernel dropped an update row since the last check.
int ctx_sync(ht_ctx* c) {
    HT_HIP(hipStreamSynchronize(c->stream));
    c->slots_all_free();
    return take_row_error(c->h_err);
}

int read_timing(hipStream_t stream, Timing& tm, double* force_ms, int64_t* launches, int64_t* pairs) {
    HT_HIP(hipStreamSynchronize(stream));
    double total = 0.0;
    for (size_t k = 0; k + 1 < tm.used; k += 2) {
        float ms = 0.0f;
        HT_HIP(hipEventElapsedTime(&ms, tm.pool[k], tm.pool[k + 1]));
        total += ms;
    }
    *force_ms = total;
    *launches = static_cast<int64_t>(tm.used / 2);
    *pairs = tm.pairs;
    tm.used = 0;
    tm.pairs = 0;
    return HT_OK;
}

// Eager mode: predict the whole combined memory into the predicted records.
int launch_predict_all(ht_ctx* c) {
    const int total = c->n + c->n_nodes;
    const Desc d = c->desc();
    const int grid = std::min((total + kWG - 1) / kWG, 8192);
    if (c->cfg.precision == HT_PREC_FP64)
        predict_all_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(d, total);
    else
        predict_all_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(d, total);
    HT_HIP(hipGetLastError());
    return HT_OK;
}

// Arguments of a device-side j-memory update (ht_set_j_particles_async).
int check_dev_rows(const ht_ctx* c, int32_t n, const int32_t* d_idx, const double* d_t0, const double* d_m,
                   const double* d_x, const double* d_v, const double* d_a, const double* d_jerk) {
    if (!c->have_particles) return fail(HT_ESTATE, "partial update before a full upload");
    if (n < 0 || n > c->n) return fail(HT_EINVAL, "n = %d outside [0, N]", n);
    const double* vec[] = {d_t0, d_m, d_x, d_v, d_a, d_jerk};
    if (n > 0 && (!d_idx || !check_vectors(vec, 6))) return fail(HT_EINVAL, "NULL device array");
    return HT_OK;
}

// Plan, pack and launch one force call on the context's stream.  Update rows
// `u` (u.n == 0: none) are written into the records by the same launch that
// delivers the plan; with `predict_eager` the whole combined memory is then
// predicted (eager mode) before the force launch.
int enqueue_step(ht_ctx* c, const DevRows& u, bool predict_eager, int32_t n_active, const int32_t* ids,
                 double* d_acc, double* d_jerk, double* d_pot, bool direct) {
    size_t end = 0;
    const int64_t* d_bins = nullptr;
    if (n_active > 0) {
        int rc = plan(c, n_active, ids, direct, true);
        if (rc) return rc;
        rc = c->slot_acquire();
        if (rc) return rc;
        Entry e{};
        end = pack_plan(c, sizeof(Entry), n_active, ids, d_acc, d_jerk, d_pot, e);
        if (direct) e.d.self_once = c->cfg.eps2 > 0.0 ? 1 : 0;   // every particle once
        if (c->n_bins > 1) {   // the placed plan's run offsets
            const size_t o_bins = align_up(end);
            std::memcpy(c->plan_host() + o_bins, c->bin_off, static_cast<size_t>(c->n_bins + 1) * 8);
            d_bins = reinterpret_cast<const int64_t*>(c->ws + c->L.off_plan + o_bins);
            end = o_bins + static_cast<size_t>(c->n_bins + 1) * 8;
        }
        e.first_item = 0;
        e.first_rtile = 0;
        e.n_items = static_cast<int64_t>(c->items.size());
        e.n_rtiles = static_cast<int64_t>(c->rtiles.size());
        std::memcpy(c->plan_host(), &e, sizeof(Entry));
    } else {
        c->last_pairs = 0;
        c->last_items = 0;
    }
    int rc = launch_prep_any(c->cfg.precision, c->stream, c->plan_host(), c->ws + c->L.off_plan, end,
                             c->ws + c->L.off_rec, u);
    if (rc) return rc;
    if (predict_eager) {
        rc = launch_predict_all(c);
        if (rc) return rc;
    }
    if (n_active == 0) return HT_OK;
    const Entry* d_tab = reinterpret_cast<const Entry*>(c->ws + c->L.off_plan);
    const int64_t ni = static_cast<int64_t>(c->items.size()), nr = static_cast<int64_t>(c->rtiles.size());
    const bool eager = c->cfg.predict_mode == HT_PREDICT_EAGER;
    const bool runs = c->list_form == HT_LISTS_RUNS && !direct;
    rc = c->cfg.precision == HT_PREC_FP64
             ? launch_force<PrecFp64>(c->stream, eager, c->tm, d_tab, 1, ni, nr, direct, c->last_pairs, runs,
                                      d_bins, c->n_bins, c->bin_max, c->union_items > 0 && !direct)
             : launch_force<PrecMixed>(c->stream, eager, c->tm, d_tab, 1, ni, nr, direct, c->last_pairs, runs,
                                       d_bins, c->n_bins, c->bin_max, c->union_items > 0 && !direct);
    if (rc) return rc;
    // The prep launch is the slot's only reader; marking the slot after the
    // whole step keeps the step's launches back to back on the host.
    return c->slot_release();
}

int force_common(ht_ctx* c, int32_t n_active, const int32_t* ids, double* d_acc, double* d_jerk, double* d_pot,
                 bool direct) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_particles) return fail(HT_ESTATE, "particles not set");
    if (!direct && !c->have_lists) return fail(HT_ESTATE, "interaction lists not set");
    if (!c->predicted) return fail(HT_ESTATE, "ht_predict not called since the last j-memory change");
    int rc = validate_active(c, n_active, ids);
    if (rc) return rc;
    if (n_active > 0 && (!d_acc || !d_jerk || !d_pot)) return fail(HT_EINVAL, "output pointer is NULL");
    return enqueue_step(c, DevRows{}, false, n_active, ids, d_acc, d_jerk, d_pot, direct);
}

int force_to_host(ht_ctx* c, int32_t n_active, const int32_t* ids, double* acc, double* jerk, double* pot,
                  bool direct) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (n_active > 0 && (!acc || !jerk || !pot)) return fail(HT_EINVAL, "output pointer is NULL");
    double* dacc = c->dev<double>(c->L.off_out);
    double* djerk = dacc + 3 * static_cast<size_t>(c->cfg.active_max);
    double* dpot = djerk + 3 * static_cast<size_t>(c->cfg.active_max);
    int rc = force_common(c, n_active, ids, dacc, djerk, dpot, direct);
    if (rc || n_active == 0) return rc;
    char* h = c->h_out;
    const size_t n3 = 3 * static_cast<size_t>(n_active) * 8, n1 = static_cast<size_t>(n_active) * 8;
    HT_HIP(hipMemcpyAsync(h, dacc, n3, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipMemcpyAsync(h + n3, djerk, n3, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipMemcpyAsync(h + 2 * n3, dpot, n1, hipMemcpyDeviceToHost, c->stream));
    rc = ctx_sync(c);
    if (rc) return rc;
    std::memcpy(acc, h, n3);
    std::memcpy(jerk, h + n3, n3);
    std::memcpy(pot, h + 2 * n3, n1);
    return HT_OK;
}

// Host rows -> device staging -> scatter kernel, in chunks.
int upload_rows(ht_ctx* c, int32_t n, const int32_t* idx, int base, const double* t0, double t0_all,
                const double* m, const double* x, const double* v, const double* a, const double* jerk) {
    char* st = c->ws + c->L.off_stage;
    int32_t* s_idx = reinterpret_cast<int32_t*>(st);
    double* s_t0 = reinterpret_cast<double*>(st + align_up(kStageRows * 4));
    double* s_m = s_t0 + kStageRows;
    double* s_x = s_m + kStageRows;
    double* s_v = s_x + 3 * kStageRows;
    double* s_a = s_v + 3 * kStageRows;
    double* s_j = s_a + 3 * kStageRows;
    const Desc d = c->desc();
    for (int32_t k0 = 0; k0 < n; k0 += kStageRows) {
        const int32_t cnt = std::min<int32_t>(kStageRows, n - k0);
        const size_t r3 = 3 * static_cast<size_t>(cnt) * 8;
        if (idx) HT_HIP(hipMemcpyAsync(s_idx, idx + k0, cnt * 4, hipMemcpyHostToDevice, c->stream));
        if (t0) HT_HIP(hipMemcpyAsync(s_t0, t0 + k0, cnt * 8, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(s_m, m + k0, cnt * 8, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(s_x, x + 3 * static_cast<size_t>(k0), r3, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(s_v, v + 3 * static_cast<size_t>(k0), r3, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(s_a, a + 3 * static_cast<size_t>(k0), r3, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(s_j, jerk + 3 * static_cast<size_t>(k0), r3, hipMemcpyHostToDevice, c->stream));
        const int grid = (cnt + kWG - 1) / kWG;
        if (c->cfg.precision == HT_PREC_FP64)
            scatter_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(d, cnt, idx ? s_idx : nullptr, base + k0,
                                                                t0 ? s_t0 : nullptr, t0_all, s_m, s_x, s_v, s_a, s_j,
                                                                c->n, c->h_err);
        else
            scatter_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(d, cnt, idx ? s_idx : nullptr, base + k0,
                                                               t0 ? s_t0 : nullptr, t0_all, s_m, s_x, s_v, s_a, s_j,
                                                                c->n, c->h_err);
        HT_HIP(hipGetLastError());
        // the staging area is reused by the next chunk: copies are ordered on the stream, and
        // pageable host sources are consumed before hipMemcpyAsync returns
    }
    return ctx_sync(c);
}

int validate_ids_unique(const ht_ctx* c, int32_t n, const int32_t* idx) {
    std::vector<uint8_t> seen(static_cast<size_t>(c->n), 0);
    for (int32_t k = 0; k < n; ++k) {
        if (idx[k] < 0 || idx[k] >= c->n) return fail(HT_ERANGE, "particle index %d outside [0, %d)", idx[k], c->n);
        if (seen[idx[k]]++) return fail(HT_EINVAL, "particle index %d repeated", idx[k]);
    }
    return HT_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// C-ABI
extern "C" {

const char* ht_last_error(void) { return g_err.c_str(); }

int ht_workspace_bytes(const ht_config* cfg, size_t* bytes) {
    if (!cfg || !bytes) return fail(HT_EINVAL, "NULL argument");
    Layout L;
    if (!layout_of(*cfg, L)) return fail(HT_EINVAL, "invalid configuration");
    *bytes = L.total;
    return HT_OK;
}

int ht_create(ht_ctx** out, const ht_config* cfg, void* d_workspace, size_t workspace_bytes) {
    if (!out || !cfg) return fail(HT_EINVAL, "NULL argument");
    *out = nullptr;
    Layout L;
    if (!layout_of(*cfg, L)) return fail(HT_EINVAL, "invalid configuration");
    if (!(cfg->eps2 >= 0.0) || !std::isfinite(cfg->eps2)) return fail(HT_EINVAL, "eps2 must be finite and >= 0");
    if (d_workspace && workspace_bytes < L.total)
        return fail(HT_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, L.total);
    if (d_workspace && (reinterpret_cast<uintptr_t>(d_workspace) & 255))
        return fail(HT_EINVAL, "workspace not 256-byte aligned");
    HT_HIP(hipSetDevice(cfg->device));
    ht_ctx* c = new ht_ctx();
    c->cfg = *cfg;
    c->L = L;
    int xcc = 1;
    if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, cfg->device) != hipSuccess || xcc < 1) xcc = 1;
    c->n_xcc = std::min(xcc, kMaxBins);
    auto cleanup = [&](int rc) {
        ht_destroy(c);
        return rc;
    };
    if (cfg->stream) {
        c->stream = static_cast<hipStream_t>(cfg->stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(HT_EHIP, "hipStreamCreateWithFlags failed"));
        c->own_stream = true;
    }
    if (d_workspace) {
        c->ws = static_cast<char*>(d_workspace);
    } else {
        if (hipMalloc(&c->ws, L.total) != hipSuccess) return cleanup(fail(HT_ENOMEM, "hipMalloc of %zu bytes failed", L.total));
        c->own_ws = true;
    }
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align_up(o + b);
        return at;
    };
    take(ht_ctx::kPlanSlots * L.plan_bytes);
    const size_t out_at = take(static_cast<size_t>(cfg->active_max) * kOut * 8);
    const size_t err_at = take(sizeof(int32_t));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_pinned), o, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(HT_ENOMEM, "hipHostMalloc of %zu bytes failed", o));
    c->h_out = c->h_pinned + out_at;
    c->h_err = reinterpret_cast<int32_t*>(c->h_pinned + err_at);
    *c->h_err = 0;
    for (int k = 0; k < ht_ctx::kPlanSlots; ++k)
        if (hipEventCreateWithFlags(&c->slot_free[k], hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(HT_EHIP, "hipEventCreate failed"));
    c->items.reserve(1024);
    tile_table(c->gather_cost, c->first_tile);
    *out = c;
    return HT_OK;
}

int ht_destroy(ht_ctx* c) {
    if (!c) return HT_OK;
    // teardown: failures here cannot be acted on, so their codes are dropped
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->slot_free)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
    for (int k = 0; k < ht_ctx::kGraphSlots; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
        if (c->hdr_free[k]) (void)hipEventDestroy(c->hdr_free[k]);
    }
    if (c->loop_exec) (void)hipGraphExecDestroy(c->loop_exec);
    if (c->loop_graph) (void)hipGraphDestroy(c->loop_graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_hdr) (void)hipHostFree(c->h_hdr);
    if (c->ds_mem && c->own_ds) (void)hipFree(c->ds_mem);
    if (c->h_dout) (void)hipHostFree(c->h_dout);
    if (c->h_active) (void)hipHostFree(c->h_active);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->d_run_start) (void)hipFree(c->d_run_start);
    if (c->d_run_pos) (void)hipFree(c->d_run_pos);
    if (c->d_copy_rec) (void)hipFree(c->d_copy_rec);
    if (c->d_copy_src) (void)hipFree(c->d_copy_src);
    if (c->d_uent) (void)hipFree(c->d_uent);
    if (c->d_umask) (void)hipFree(c->d_umask);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return HT_OK;
}

int ht_set_j_particles(ht_ctx* c, int32_t n, const int32_t* idx, const double* t0, const double* m,
                       const double* x, const double* v, const double* a, const double* jerk) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    const double* vec[] = {t0, m, x, v, a, jerk};
    if (n < 0) return fail(HT_EINVAL, "n < 0");
    if (n > 0 && !check_vectors(vec, 6)) return fail(HT_EINVAL, "NULL particle array");
    if (!idx) {
        if (n < 1) return fail(HT_EINVAL, "full upload needs n >= 1");
        if (n > c->cfg.n_max) return fail(HT_ERANGE, "n = %d over capacity %d", n, c->cfg.n_max);
        if (n != c->n) {
            c->have_nodes = false;
            c->have_lists = false;
            c->n_nodes = 0;
        }
        int rc = upload_rows(c, n, nullptr, 0, t0, 0.0, m, x, v, a, jerk);
        if (rc) return rc;
        c->n = n;
        c->have_particles = true;
    } else {
        if (!c->have_particles) return fail(HT_ESTATE, "partial update before a full upload");
        int rc = validate_ids_unique(c, n, idx);
        if (rc) return rc;
        if (n == 0) return HT_OK;
        rc = upload_rows(c, n, idx, 0, t0, 0.0, m, x, v, a, jerk);
        if (rc) return rc;
    }
    c->predicted = false;
    return HT_OK;
}

int ht_set_j_particles_async(ht_ctx* c, int32_t n, const int32_t* d_idx, const double* d_t0, const double* d_m,
                             const double* d_x, const double* d_v, const double* d_a, const double* d_jerk) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    int rc = check_dev_rows(c, n, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk);
    if (rc) return rc;
    c->predicted = false;
    if (n == 0) return HT_OK;
    const Desc d = c->desc();
    const int grid = (n + kWG - 1) / kWG;
    if (c->cfg.precision == HT_PREC_FP64)
        scatter_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(d, n, d_idx, 0, d_t0, 0.0, d_m, d_x, d_v, d_a, d_jerk,
                                                            c->n, c->h_err);
    else
        scatter_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(d, n, d_idx, 0, d_t0, 0.0, d_m, d_x, d_v, d_a, d_jerk,
                                                            c->n, c->h_err);
    HT_HIP(hipGetLastError());
    return HT_OK;
}

int ht_set_nodes(ht_ctx* c, int32_t n_nodes, double t_tree, const double* m, const double* x, const double* v,
                 const double* a, const double* jerk) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_particles) return fail(HT_ESTATE, "nodes before particles");
    if (n_nodes < 0 || n_nodes > c->cfg.node_max)
        return fail(HT_ERANGE, "n_nodes = %d outside [0, %d]", n_nodes, c->cfg.node_max);
    const double* vec[] = {m, x, v, a, jerk};
    if (n_nodes > 0 && !check_vectors(vec, 5)) return fail(HT_EINVAL, "NULL node array");
    if (!std::isfinite(t_tree)) return fail(HT_EINVAL, "t_tree not finite");
    if (n_nodes > 0) {
        int rc = upload_rows(c, n_nodes, nullptr, c->n, nullptr, t_tree, m, x, v, a, jerk);
        if (rc) return rc;
    }
    c->n_nodes = n_nodes;
    c->have_nodes = true;
    c->have_lists = false;
    c->predicted = false;
    return HT_OK;
}

namespace {
int upload_group_offsets(ht_ctx* c);

// Run-length form of the lists just set (Section 2's cell-index memory of
// start and count pairs, with each group's nodes copied contiguously): the
// node entries of every list, in list order, are replaced by copies of their
// records at consecutive indices from N + M on, and the list becomes runs of
// consecutive indices (Peano-Hilbert order makes neighbouring particles
// neighbouring indices).  Expanded, the runs give back the lists' records in
// the lists' order, so the force is the CSR form's, bit for bit.
int build_runs(ht_ctx* c, const int32_t* entries) {
    const int64_t L = c->list_off.back();
    const int64_t base = static_cast<int64_t>(c->n) + c->n_nodes;
    std::vector<int32_t> start, src;
    std::vector<int64_t> pos;
    int64_t prev = -2;
    for (int64_t e = 0; e < L; ++e) {
        const int32_t j = entries[e];
        int64_t idx = j;
        if (j >= c->n) {
            idx = base + static_cast<int64_t>(src.size());
            src.push_back(j);
        }
        if (idx != prev + 1) {
            start.push_back(static_cast<int32_t>(idx));
            pos.push_back(e);
        }
        prev = idx;
    }
    if (base + static_cast<int64_t>(src.size()) > INT32_MAX)
        return fail(HT_ERANGE, "%zu node copies do not fit 32-bit indices", src.size());
    const size_t nr = start.size(), nc = src.size();
    if (nr > c->run_cap) {
        if (c->d_run_start) (void)hipFree(c->d_run_start);
        if (c->d_run_pos) (void)hipFree(c->d_run_pos);
        c->d_run_start = nullptr;
        c->d_run_pos = nullptr;
        c->run_cap = 0;
        if (hipMalloc(&c->d_run_start, nr * 4) != hipSuccess || hipMalloc(&c->d_run_pos, nr * 8) != hipSuccess)
            return fail(HT_ENOMEM, "hipMalloc of %zu runs failed", nr);
        c->run_cap = nr;
    }
    if (nc > c->copy_cap) {
        if (c->d_copy_rec) (void)hipFree(c->d_copy_rec);
        if (c->d_copy_src) (void)hipFree(c->d_copy_src);
        c->d_copy_rec = nullptr;
        c->d_copy_src = nullptr;
        c->copy_cap = 0;
        if (hipMalloc(&c->d_copy_rec, nc * 128) != hipSuccess || hipMalloc(&c->d_copy_src, nc * 4) != hipSuccess)
            return fail(HT_ENOMEM, "hipMalloc of %zu node copies failed", nc);
        c->copy_cap = nc;
    }
    if (nr) {
        HT_HIP(hipMemcpyAsync(c->d_run_start, start.data(), nr * 4, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(c->d_run_pos, pos.data(), nr * 8, hipMemcpyHostToDevice, c->stream));
    }
    if (nc) {
        HT_HIP(hipMemcpyAsync(c->d_copy_src, src.data(), nc * 4, hipMemcpyHostToDevice, c->stream));
        const int grid = static_cast<int>(std::min<size_t>((nc + kWG - 1) / kWG, 65536));
        const void* rec = c->ws + c->L.off_rec;
        if (c->cfg.precision == HT_PREC_FP64)
            copy_records_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(rec, c->d_copy_src, static_cast<int64_t>(nc),
                                                                       c->d_copy_rec);
        else
            copy_records_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(rec, c->d_copy_src, static_cast<int64_t>(nc),
                                                                        c->d_copy_rec);
        HT_HIP(hipGetLastError());
    }
    c->run_pos = std::move(pos);
    c->n_runs = static_cast<int64_t>(nr);
    c->n_copies = static_cast<int64_t>(nc);
    return ctx_sync(c);   // pageable sources
}
// Union tiles: the groups in runs of union_width consecutive groups; each run's
// union list holds every entry of its members' lists once, in order of first
// appearance over the members in group order, with a bit per member whose list
// holds it.  Host work linear in the lists' length.
int build_unions(ht_ctx* c, int32_t n_groups, const int64_t* list_off, const int32_t* entries) {
    const int32_t w = c->union_width;
    const int32_t n_runs = (n_groups + w - 1) / w;
    std::vector<int32_t> ue;
    std::vector<uint8_t> um;
    ue.reserve(static_cast<size_t>(list_off[n_groups]));
    um.reserve(static_cast<size_t>(list_off[n_groups]));
    std::vector<int64_t> pos(static_cast<size_t>(c->n) + c->n_nodes, -1);
    c->u_off.assign(static_cast<size_t>(n_runs) + 1, 0);
    for (int32_t r = 0; r < n_runs; ++r) {
        const size_t start = ue.size();
        for (int32_t q = 0; q < w && r * w + q < n_groups; ++q) {
            const int32_t g = r * w + q;
            for (int64_t e = list_off[g]; e < list_off[g + 1]; ++e) {
                const int32_t j = entries[e];
                if (pos[j] < 0) {
                    pos[j] = static_cast<int64_t>(ue.size());
                    ue.push_back(j);
                    um.push_back(static_cast<uint8_t>(1u << q));
                } else {
                    um[pos[j]] = static_cast<uint8_t>(um[pos[j]] | (1u << q));
                }
            }
        }
        for (size_t k = start; k < ue.size(); ++k) pos[ue[k]] = -1;
        c->u_off[r + 1] = static_cast<int64_t>(ue.size());
    }
    const size_t nu = ue.size();
    if (nu > c->ucap) {
        if (c->d_uent) (void)hipFree(c->d_uent);
        if (c->d_umask) (void)hipFree(c->d_umask);
        c->d_uent = nullptr;
        c->d_umask = nullptr;
        c->ucap = 0;
        if (hipMalloc(&c->d_uent, nu * 4) != hipSuccess || hipMalloc(&c->d_umask, nu) != hipSuccess)
            return fail(HT_ENOMEM, "hipMalloc of %zu union entries failed", nu);
        c->ucap = nu;
    }
    if (nu) {
        HT_HIP(hipMemcpyAsync(c->d_uent, ue.data(), nu * 4, hipMemcpyHostToDevice, c->stream));
        HT_HIP(hipMemcpyAsync(c->d_umask, um.data(), nu, hipMemcpyHostToDevice, c->stream));
    }
    return ctx_sync(c);   // pageable sources
}

}  // namespace

int ht_set_interaction_lists(ht_ctx* c, int32_t n_groups, const int64_t* group_first, const int64_t* list_off,
                             const int32_t* entries) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_particles || !c->have_nodes) return fail(HT_ESTATE, "lists before particles and nodes");
    if (n_groups < 1 || n_groups > c->cfg.group_max)
        return fail(HT_ERANGE, "n_groups = %d outside [1, %d]", n_groups, c->cfg.group_max);
    if (!group_first || !list_off) return fail(HT_EINVAL, "NULL group array");
    if (group_first[0] != 0 || group_first[n_groups] != c->n)
        return fail(HT_EINVAL, "group_first must run from 0 to N = %d", c->n);
    for (int32_t g = 0; g < n_groups; ++g)
        if (group_first[g + 1] <= group_first[g]) return fail(HT_EINVAL, "group_first not strictly increasing at %d", g);
    if (list_off[0] != 0) return fail(HT_EINVAL, "list_off[0] != 0");
    for (int32_t g = 0; g < n_groups; ++g)
        if (list_off[g + 1] < list_off[g]) return fail(HT_EINVAL, "list_off decreasing at %d", g);
    const int64_t L = list_off[n_groups];
    if (L > c->cfg.list_max) return fail(HT_ERANGE, "%lld list entries over capacity %lld", (long long)L,
                                         (long long)c->cfg.list_max);
    if (L > 0 && !entries) return fail(HT_EINVAL, "entries is NULL");
    const int32_t jmax = c->n + c->n_nodes;
    for (int64_t e = 0; e < L; ++e)
        if (entries[e] < 0 || entries[e] >= jmax)
            return fail(HT_ERANGE, "entry %lld = %d outside [0, %d)", (long long)e, entries[e], jmax);
    if (L > 0) {
        HT_HIP(hipMemcpyAsync(c->ws + c->L.off_entries, entries, static_cast<size_t>(L) * 4, hipMemcpyHostToDevice,
                              c->stream));
        int rc = ctx_sync(c);
        if (rc) return rc;
    }
    c->group_first.assign(group_first, group_first + n_groups + 1);
    c->list_off.assign(list_off, list_off + n_groups + 1);
    c->n_groups = n_groups;
    c->n_entries = L;
    {   // does every list hold each particle of its group exactly once?
        std::vector<uint8_t> seen(static_cast<size_t>(c->n), 0);
        bool once = true;
        for (int32_t g = 0; g < n_groups && once; ++g)
            for (int64_t e = list_off[g]; e < list_off[g + 1]; ++e) {
                const int32_t j = entries[e];
                if (j >= group_first[g] && j < group_first[g + 1] && seen[j]++) {
                    once = false;
                    break;
                }
            }
        for (int32_t k = 0; k < c->n && once; ++k) once = seen[k] == 1;
        c->self_once_lists = once;
    }
    if (c->list_form == HT_LISTS_RUNS) {
        int rc = build_runs(c, entries);
        if (rc) return rc;
    }
    if (c->list_form == HT_LISTS_UNION) {
        int rc = build_unions(c, n_groups, list_off, entries);
        if (rc) return rc;
    }
    c->have_lists = true;
    if (c->ds_mem) return upload_group_offsets(c);
    return HT_OK;
}

int ht_predict(ht_ctx* c, double t) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_particles) return fail(HT_ESTATE, "predict before particles");
    if (!std::isfinite(t)) return fail(HT_EINVAL, "t not finite");
    c->t_pred = t;
    if (c->cfg.predict_mode == HT_PREDICT_EAGER) {
        int rc = launch_predict_all(c);
        if (rc) return rc;
    }
    c->predicted = true;
    return HT_OK;
}

int ht_predict_many(int32_t n_ctx, ht_ctx* const* ctxs, const double* t) {
    if (n_ctx < 0 || (n_ctx > 0 && (!ctxs || !t))) return fail(HT_EINVAL, "bad arguments");
    for (int32_t k = 0; k < n_ctx; ++k) {
        if (!ctxs[k]) return fail(HT_EINVAL, "ctx %d is NULL", k);
        if (!ctxs[k]->have_particles) return fail(HT_ESTATE, "ctx %d: predict before particles", k);
        if (!std::isfinite(t[k])) return fail(HT_EINVAL, "ctx %d: t not finite", k);
    }
    for (int32_t k = 0; k < n_ctx; ++k) {
        int rc = ht_predict(ctxs[k], t[k]);
        if (rc) return rc;
    }
    return HT_OK;
}

int ht_set_list_form(ht_ctx* c, int32_t form) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (form != HT_LISTS_CSR && form != HT_LISTS_RUNS && form != HT_LISTS_UNION)
        return fail(HT_EINVAL, "unknown list form %d", form);
    if (form != HT_LISTS_CSR && c->cfg.predict_mode != HT_PREDICT_FUSED)
        return fail(HT_EINVAL, "run-length lists and union tiles need fused prediction");
    if (form != c->list_form) {
        c->list_form = form;
        c->have_lists = false;   // the lists must be set again, in the new form
    }
    return HT_OK;
}

int ht_set_union_width(ht_ctx* c, int32_t width) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (width < 2 || width > 8) return fail(HT_EINVAL, "union width %d outside [2, 8]", width);
    if (width != c->union_width) {
        c->union_width = width;
        if (c->list_form == HT_LISTS_UNION) c->have_lists = false;   // set the lists again
    }
    return HT_OK;
}

int ht_force(ht_ctx* c, int32_t n_active, const int32_t* ids, double* acc, double* jerk, double* pot) {
    return force_to_host(c, n_active, ids, acc, jerk, pot, false);
}

int ht_force_async(ht_ctx* c, int32_t n_active, const int32_t* ids, double* d_acc, double* d_jerk, double* d_pot) {
    return force_common(c, n_active, ids, d_acc, d_jerk, d_pot, false);
}

int ht_force_direct(ht_ctx* c, int32_t n_active, const int32_t* ids, double* acc, double* jerk, double* pot) {
    return force_to_host(c, n_active, ids, acc, jerk, pot, true);
}

int ht_force_direct_async(ht_ctx* c, int32_t n_active, const int32_t* ids, double* d_acc, double* d_jerk,
                          double* d_pot) {
    return force_common(c, n_active, ids, d_acc, d_jerk, d_pot, true);
}

int ht_step_async(ht_ctx* c, int32_t n_upd, const int32_t* d_idx, const double* d_t0, const double* d_m,
                  const double* d_x, const double* d_v, const double* d_a, const double* d_jerk, double t,
                  int32_t n_active, const int32_t* ids, double* d_acc, double* d_jerk_out, double* d_pot) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_lists) return fail(HT_ESTATE, "interaction lists not set");
    int rc = check_dev_rows(c, n_upd, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk);
    if (rc) return rc;
    rc = validate_active(c, n_active, ids);
    if (rc) return rc;
    if (!std::isfinite(t)) return fail(HT_EINVAL, "t not finite");
    if (n_active > 0 && (!d_acc || !d_jerk_out || !d_pot)) return fail(HT_EINVAL, "output pointer is NULL");
    c->t_pred = t;
    c->predicted = true;
    const DevRows u{n_upd, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk, c->n, c->h_err};
    return enqueue_step(c, u, c->cfg.predict_mode == HT_PREDICT_EAGER, n_active, ids, d_acc, d_jerk_out, d_pot,
                        false);
}

}  // extern "C"

namespace {

// The scheduler's table entry of a context whose blocks start at first_block.
SchedEntry sched_entry_of(const ht_ctx* c, int32_t first_block) {
    const int64_t n = c->n;
    const int nb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(kSchedBlocks, (n + 2047) / 2048)));
    return SchedEntry{c->ds.t0, c->ds.dt, c->ds.active, c->ds.bmin, c->ds.bcount, n, (n + nb - 1) / nb, nb,
                      first_block, c->h_dout, c->h_active, nullptr};
}

// The corrector's table entry of a context's last active set, rows from first_row.
CorrEntry corr_entry_of(const ht_ctx* c, int64_t first_row, double eta, double dt_tree) {
    return CorrEntry{c->ds, c->ws + c->L.off_rec, c->h_dout, c->dev_n_active, first_row, c->dev_t_next, eta, dt_tree,
                     nullptr, nullptr, nullptr, nullptr};
}

int launch_correct(int precision, hipStream_t stream, const CorrEntry& e0, const CorrEntry* tab, int n_tab,
                   int64_t total) {
    const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((total + kWG - 1) / kWG, 65536)));
    if (precision == HT_PREC_FP64)
        dev_correct_kernel<PrecFp64><<<grid, kWG, 0, stream>>>(e0, tab, n_tab, total, nullptr);
    else
        dev_correct_kernel<PrecMixed><<<grid, kWG, 0, stream>>>(e0, tab, n_tab, total, nullptr);
    HT_HIP(hipGetLastError());
    return HT_OK;
}

constexpr int kGraphForceGrid = 2048;   // fixed force grid of a replay (2 per resident work-group slot)
constexpr int kGraphCopyBlocks = 256;
constexpr int kGraphScatterBlocks = 256;
constexpr int kGraphReduceGrid = 256;

// Capture the step graph of header slot k: prep (plan pulled from the
// header's slot, update rows written), force and reduce (fixed grids, counts
// read from the plan).
template <class P>
int build_step_graph(ht_ctx* c, int k) {
    if (!c->cap_stream) HT_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->h_hdr) {
        HT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_hdr), ht_ctx::kGraphSlots * sizeof(GraphHdr),
                             hipHostMallocDefault));
        std::memset(c->h_hdr, 0, ht_ctx::kGraphSlots * sizeof(GraphHdr));
        for (int q = 0; q < ht_ctx::kGraphSlots; ++q)
            HT_HIP(hipEventCreateWithFlags(&c->hdr_free[q], hipEventDisableTiming));
    }
    uint64_t* d_plan = reinterpret_cast<uint64_t*>(c->ws + c->L.off_plan);
    const Entry* d_tab = reinterpret_cast<const Entry*>(c->ws + c->L.off_plan);
    hipStream_t s = c->cap_stream;
    HT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    prep_graph_kernel<P><<<kGraphCopyBlocks + kGraphScatterBlocks, kWG, 0, s>>>(c->h_hdr + k, d_plan,
                                                                             c->ws + c->L.off_rec,
                                                                             kGraphCopyBlocks);
    force_kernel<P, false, false><<<kGraphForceGrid, kWG, 0, s>>>(d_tab, 1, -1, &d_tab->n_items);
    reduce_kernel<<<kGraphReduceGrid, kWG, 0, s>>>(d_tab, 1, -1);
    const hipError_t launch = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(s, &g);
    if (launch != hipSuccess || end != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(HT_EHIP, "capturing the step graph failed: %s",
                    hipGetErrorString(launch != hipSuccess ? launch : end));
    }
    c->graph[k] = g;
    HT_HIP(hipGraphInstantiate(&c->gexec[k], g, nullptr, nullptr, 0));
    return HT_OK;
}

}  // namespace

extern "C" {

int ht_step_graph(ht_ctx* c, int32_t n_upd, const int32_t* d_idx, const double* d_t0, const double* d_m,
                  const double* d_x, const double* d_v, const double* d_a, const double* d_jerk, double t,
                  int32_t n_active, const int32_t* ids, double* d_acc, double* d_jerk_out, double* d_pot) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (c->cfg.predict_mode != HT_PREDICT_FUSED) return fail(HT_EINVAL, "graph steps need fused prediction");
    if (c->list_form != HT_LISTS_CSR) return fail(HT_EINVAL, "graph steps take CSR lists");
    if (!c->have_lists) return fail(HT_ESTATE, "interaction lists not set");
    int rc = check_dev_rows(c, n_upd, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk);
    if (rc) return rc;
    rc = validate_active(c, n_active, ids);
    if (rc) return rc;
    if (!std::isfinite(t)) return fail(HT_EINVAL, "t not finite");
    if (n_active > 0 && (!d_acc || !d_jerk_out || !d_pot)) return fail(HT_EINVAL, "output pointer is NULL");
    if (n_active == 0) {   // nothing to replay: the update alone, as ht_step_async would do it
        const DevRows u{n_upd, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk, c->n, c->h_err};
        c->t_pred = t;
        c->predicted = true;
        return enqueue_step(c, u, false, 0, ids, d_acc, d_jerk_out, d_pot, false);
    }
    c->t_pred = t;
    c->predicted = true;
    rc = plan(c, n_active, ids, false);
    if (rc) return rc;
    rc = c->slot_acquire();
    if (rc) return rc;
    Entry e{};
    const size_t end = pack_plan(c, sizeof(Entry), n_active, ids, d_acc, d_jerk_out, d_pot, e);
    e.first_item = 0;
    e.first_rtile = 0;
    e.n_items = static_cast<int64_t>(c->items.size());
    e.n_rtiles = static_cast<int64_t>(c->rtiles.size());
    std::memcpy(c->plan_host(), &e, sizeof(Entry));
    const int k = c->gslot;
    if (!c->gexec[k]) {
        rc = c->cfg.precision == HT_PREC_FP64 ? build_step_graph<PrecFp64>(c, k) : build_step_graph<PrecMixed>(c, k);
        if (rc) return rc;
    }
    if (c->hdr_pending[k]) {
        HT_HIP(hipEventSynchronize(c->hdr_free[k]));
        c->hdr_pending[k] = false;
    }
    GraphHdr& h = c->h_hdr[k];
    h.n8 = static_cast<int64_t>((end + 7) / 8);
    h.src = reinterpret_cast<const uint64_t*>(c->plan_host());
    h.n_upd = n_upd;
    h.idx = d_idx;
    h.t0 = d_t0;
    h.m = d_m;
    h.x = d_x;
    h.v = d_v;
    h.a = d_a;
    h.jerk = d_jerk;
    h.lim = c->n;
    h.err = c->h_err;
    Timing& tm = c->tm;
    if (tm.enabled) {
        while (tm.pool.size() < tm.used + 2) {
            hipEvent_t ev;
            HT_HIP(hipEventCreate(&ev));
            tm.pool.push_back(ev);
        }
        HT_HIP(hipEventRecord(tm.pool[tm.used], c->stream));
    }
    HT_HIP(hipGraphLaunch(c->gexec[k], c->stream));
    if (tm.enabled) {
        HT_HIP(hipEventRecord(tm.pool[tm.used + 1], c->stream));
        tm.used += 2;
        tm.pairs += c->last_pairs;
    }
    HT_HIP(hipEventRecord(c->hdr_free[k], c->stream));
    c->hdr_pending[k] = true;
    c->gslot = (k + 1) % ht_ctx::kGraphSlots;
    return c->slot_release();
}

// ------------------------------------------------------------------------------------------------
// device-resident integration
namespace {
// The group and list offsets for the device planner (resident state only).
int upload_group_offsets(ht_ctx* c) {
    const size_t b = (static_cast<size_t>(c->n_groups) + 1) * 8;
    HT_HIP(hipMemcpyAsync(c->d_gfirst, c->group_first.data(), b, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->d_loff, c->list_off.data(), b, hipMemcpyHostToDevice, c->stream));
    group_of_kernel<<<(c->n + kWG - 1) / kWG, kWG, 0, c->stream>>>(c->n, c->d_gfirst, c->n_groups, c->d_pgroup);
    HT_HIP(hipGetLastError());
    return ctx_sync(c);   // pageable sources
}
}  // namespace

}  // extern "C"

namespace {

// Where the resident state's arrays sit in its one device allocation.
struct StateLayout {
    size_t x, v, a, j, t0, dt, m, pot, acc, jerk, fpot, act, bmin, bcnt;
    size_t loop, dout, gf, lo, gk, qk, qg, tiles, pgroup;
    size_t total;
};

StateLayout state_layout(const ht_config& cfg) {
    const size_t n = static_cast<size_t>(cfg.n_max);
    StateLayout S{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    S.x = take(n * 24);
    S.v = take(n * 24);
    S.a = take(n * 24);
    S.j = take(n * 24);
    S.t0 = take(n * 8);
    S.dt = take(n * 8);
    S.m = take(n * 8);
    S.pot = take(n * 8);
    S.acc = take(n * 24);
    S.jerk = take(n * 24);
    S.fpot = take(n * 8);
    S.act = take(n * 4);
    S.bmin = take(kSchedBlocks * 8);
    S.bcnt = take(kSchedBlocks * 4);
    const size_t g1 = static_cast<size_t>(cfg.group_max) + 1;
    S.loop = take(sizeof(DevLoop));
    S.dout = take(sizeof(DevOut));
    S.gf = take(g1 * 8);
    S.lo = take(g1 * 8);
    S.gk = take(n * 4);
    S.qk = take((n + 1) * 4);
    S.qg = take(n * 4);
    S.tiles = take(n * sizeof(DTile));
    S.pgroup = take(n * 4);
    S.total = o;
    return S;
}

// Point the context's resident state at `mem` (laid out by state_layout) and
// allocate its pinned scheduler results.
int state_attach(ht_ctx* c, char* mem, bool own) {
    const StateLayout S = state_layout(c->cfg);
    c->ds_mem = mem;
    c->own_ds = own;
    char* b = mem;
    c->ds = DevState{reinterpret_cast<double*>(b + S.x), reinterpret_cast<double*>(b + S.v),
                     reinterpret_cast<double*>(b + S.a), reinterpret_cast<double*>(b + S.j),
                     reinterpret_cast<double*>(b + S.t0), reinterpret_cast<double*>(b + S.dt),
                     reinterpret_cast<double*>(b + S.m), reinterpret_cast<double*>(b + S.pot),
                     reinterpret_cast<double*>(b + S.acc), reinterpret_cast<double*>(b + S.jerk),
                     reinterpret_cast<double*>(b + S.fpot), reinterpret_cast<int32_t*>(b + S.act),
                     reinterpret_cast<double*>(b + S.bmin), reinterpret_cast<int32_t*>(b + S.bcnt)};
    c->d_loop = reinterpret_cast<DevLoop*>(b + S.loop);
    c->d_dout = reinterpret_cast<DevOut*>(b + S.dout);
    c->d_gfirst = reinterpret_cast<int64_t*>(b + S.gf);
    c->d_loff = reinterpret_cast<int64_t*>(b + S.lo);
    c->d_gk = reinterpret_cast<int32_t*>(b + S.gk);
    c->d_qk = reinterpret_cast<int32_t*>(b + S.qk);
    c->d_qg = reinterpret_cast<int32_t*>(b + S.qg);
    c->d_tiles = reinterpret_cast<DTile*>(b + S.tiles);
    c->d_pgroup = reinterpret_cast<int32_t*>(b + S.pgroup);
    if (c->have_lists) {   // lists set before the state: their offsets for the device planner
        int rc = upload_group_offsets(c);
        if (rc) return rc;
    }
    const size_t n = static_cast<size_t>(c->cfg.n_max);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_dout), sizeof(DevOut), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_active), n * 4, hipHostMallocDefault) != hipSuccess)
        return fail(HT_ENOMEM, "hipHostMalloc for the scheduler results failed");
    std::memset(c->h_dout, 0, sizeof(DevOut));
    return HT_OK;
}

}  // namespace

extern "C" {

int ht_state_bytes(const ht_config* cfg, size_t* bytes) {
    if (!cfg || !bytes) return fail(HT_EINVAL, "NULL argument");
    Layout L;
    if (!layout_of(*cfg, L)) return fail(HT_EINVAL, "invalid configuration");
    *bytes = state_layout(*cfg).total;
    return HT_OK;
}

int ht_state_enable(ht_ctx* c) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (c->ds_mem) return HT_OK;
    const size_t bytes = state_layout(c->cfg).total;
    char* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(HT_ENOMEM, "hipMalloc of %zu bytes for the device state failed", bytes);
    return state_attach(c, mem, true);
}

int ht_state_enable_ws(ht_ctx* c, void* d_mem, size_t bytes) {
    if (!c || !d_mem) return fail(HT_EINVAL, "NULL argument");
    if (c->ds_mem) return fail(HT_ESTATE, "the device state is already enabled");
    const size_t need = state_layout(c->cfg).total;
    if (bytes < need) return fail(HT_EINVAL, "state memory of %zu bytes is smaller than the %zu needed", bytes, need);
    if (reinterpret_cast<uintptr_t>(d_mem) & 255) return fail(HT_EINVAL, "state memory not 256-byte aligned");
    return state_attach(c, static_cast<char*>(d_mem), false);
}

int ht_state_set(ht_ctx* c, int32_t n, const double* t0, const double* dt, const double* m, const double* x,
                 const double* v, const double* a, const double* jerk, const double* pot) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    const double* vec[] = {t0, dt, m, x, v, a, jerk};
    if (n < 1 || !check_vectors(vec, 7)) return fail(HT_EINVAL, "bad state arrays");
    int rc = ht_set_j_particles(c, n, nullptr, t0, m, x, v, a, jerk);   // the j-records
    if (rc) return rc;
    const size_t n1 = static_cast<size_t>(n) * 8, n3 = 3 * n1;
    HT_HIP(hipMemcpyAsync(c->ds.t0, t0, n1, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.dt, dt, n1, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.m, m, n1, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.x, x, n3, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.v, v, n3, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.a, a, n3, hipMemcpyHostToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.j, jerk, n3, hipMemcpyHostToDevice, c->stream));
    if (pot) HT_HIP(hipMemcpyAsync(c->ds.pot, pot, n1, hipMemcpyHostToDevice, c->stream));
    else HT_HIP(hipMemsetAsync(c->ds.pot, 0, n1, c->stream));
    c->dev_n_active = -1;
    rc = ctx_sync(c);   // pageable sources
    if (rc) return rc;
    return HT_OK;
}

int ht_state_get(ht_ctx* c, double* t0, double* dt, double* x, double* v, double* a, double* jerk, double* pot) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    const size_t n1 = static_cast<size_t>(c->n) * 8, n3 = 3 * n1;
    const struct { double* dst; const double* src; size_t bytes; } cp[] = {
        {t0, c->ds.t0, n1}, {dt, c->ds.dt, n1}, {x, c->ds.x, n3}, {v, c->ds.v, n3},
        {a, c->ds.a, n3}, {jerk, c->ds.j, n3}, {pot, c->ds.pot, n1}};
    for (const auto& k : cp)
        if (k.dst) HT_HIP(hipMemcpyAsync(k.dst, k.src, k.bytes, hipMemcpyDeviceToHost, c->stream));
    return ctx_sync(c);
}

int ht_state_rebuild(ht_ctx* c, htd_tree* t, int32_t n_leaf, int32_t n_crit, double theta, double t_tree,
                     int64_t* perm) {
    if (!c || !t) return fail(HT_EINVAL, "NULL argument");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    if (c->n < 1) return fail(HT_ESTATE, "particles not set");
    if (!std::isfinite(t_tree)) return fail(HT_EINVAL, "t_tree not finite");
    if (c->list_form != HT_LISTS_CSR) return fail(HT_EINVAL, "device rebuilds write CSR lists");
    const int32_t n = c->n;
    if (int rc = ctx_sync(c)) return rc;   // the state is complete before the builder reads it
    if (int rc = htd_build(t, n, c->ds.x, c->ds.v, c->ds.a, c->ds.j, c->ds.m, n_leaf, n_crit, theta))
        return fail(rc == HTD_EINVAL ? HT_EINVAL : rc == HTD_ENOMEM ? HT_ENOMEM : HT_EHIP, "device tree build: %s",
                    htd_last_error());
    int64_t M = 0, G = 0, L = 0;
    htd_view w{};
    if (htd_sizes(t, &M, &G, &L, nullptr) || htd_device_view(t, &w)) return fail(HT_EHIP, "%s", htd_last_error());
    if (M > c->cfg.node_max || G > c->cfg.group_max || L > c->cfg.list_max)
        return fail(HT_ERANGE, "tree needs %lld nodes, %lld groups, %lld list entries; capacity %d, %d, %lld",
                    (long long)M, (long long)G, (long long)L, c->cfg.node_max, c->cfg.group_max,
                    (long long)c->cfg.list_max);
    // the state in the new particle order: x, v, a, jerk, m come sorted from the builder;
    // dt and pot are gathered through the permutation; every t0 is the tree time
    const size_t n1 = static_cast<size_t>(n) * 8, n3 = 3 * n1;
    const int grid = (n + kWG - 1) / kWG;
    permute2_kernel<<<grid, kWG, 0, c->stream>>>(n, w.perm, c->ds.dt, c->ds.pot, c->ds.acc, c->ds.fpot);
    HT_HIP(hipGetLastError());
    HT_HIP(hipMemcpyAsync(c->ds.dt, c->ds.acc, n1, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.pot, c->ds.fpot, n1, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.x, w.x, n3, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.v, w.v, n3, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.a, w.a, n3, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.j, w.jerk, n3, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->ds.m, w.m, n1, hipMemcpyDeviceToDevice, c->stream));
    fill_kernel<<<grid, kWG, 0, c->stream>>>(n, c->ds.t0, t_tree);
    HT_HIP(hipGetLastError());
    // records: particles, then nodes at the tree time; then the lists
    const Desc d = c->desc();
    const int gn = (static_cast<int>(M) + kWG - 1) / kWG;
    if (c->cfg.precision == HT_PREC_FP64) {
        scatter_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(d, n, nullptr, 0, nullptr, t_tree, c->ds.m, c->ds.x,
                                                            c->ds.v, c->ds.a, c->ds.j, n, c->h_err);
        if (M > 0)
            scatter_kernel<PrecFp64><<<gn, kWG, 0, c->stream>>>(d, static_cast<int>(M), nullptr, n, nullptr, t_tree,
                                                              w.node_m, w.node_x, w.node_v, w.node_a, w.node_j,
                                                              n, c->h_err);
    } else {
        scatter_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(d, n, nullptr, 0, nullptr, t_tree, c->ds.m, c->ds.x,
                                                             c->ds.v, c->ds.a, c->ds.j, n, c->h_err);
        if (M > 0)
            scatter_kernel<PrecMixed><<<gn, kWG, 0, c->stream>>>(d, static_cast<int>(M), nullptr, n, nullptr, t_tree,
                                                               w.node_m, w.node_x, w.node_v, w.node_a, w.node_j,
                                                              n, c->h_err);
    }
    HT_HIP(hipGetLastError());
    HT_HIP(hipMemcpyAsync(c->ws + c->L.off_entries, w.entries, static_cast<size_t>(L) * 4, hipMemcpyDeviceToDevice,
                          c->stream));
    c->group_first.resize(static_cast<size_t>(G) + 1);
    c->list_off.resize(static_cast<size_t>(G) + 1);
    HT_HIP(hipMemcpyAsync(c->group_first.data(), w.group_first, (G + 1) * 8, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipMemcpyAsync(c->list_off.data(), w.list_off, (G + 1) * 8, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipMemcpyAsync(c->d_gfirst, w.group_first, (G + 1) * 8, hipMemcpyDeviceToDevice, c->stream));
    HT_HIP(hipMemcpyAsync(c->d_loff, w.list_off, (G + 1) * 8, hipMemcpyDeviceToDevice, c->stream));
    group_of_kernel<<<grid, kWG, 0, c->stream>>>(n, c->d_gfirst, static_cast<int32_t>(G), c->d_pgroup);
    HT_HIP(hipGetLastError());
    if (perm) HT_HIP(hipMemcpyAsync(perm, w.perm, n1, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipStreamSynchronize(c->stream));
    c->n_nodes = static_cast<int32_t>(M);
    c->n_groups = static_cast<int32_t>(G);
    c->n_entries = L;
    c->have_nodes = true;
    c->have_lists = true;
    c->self_once_lists = true;   // the builder lists every particle of a group in its list once
    c->predicted = false;
    c->dev_n_active = -1;
    return HT_OK;
}

int ht_dev_next_block(ht_ctx* c, double* t_next, int64_t* n_active, const int32_t** active) {
    if (!c || !t_next || !n_active || !active) return fail(HT_EINVAL, "NULL argument");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    if (c->n < 1) return fail(HT_ESTATE, "particles not set");
    const SchedEntry e = sched_entry_of(c, 0);
    sched_min_kernel<<<e.nb, kWG, 0, c->stream>>>(e, nullptr, 0);
    sched_count_kernel<<<e.nb, kWG, 0, c->stream>>>(e, nullptr, 0);
    sched_write_kernel<<<e.nb, kWG, 0, c->stream>>>(e, nullptr, 0);
    HT_HIP(hipGetLastError());
    if (int rc = ctx_sync(c)) return rc;
    if (c->h_dout->below_floor) {
        c->h_dout->below_floor = 0;
        return fail(HT_ERANGE, "a corrected block step fell below 2^-40");
    }
    c->dev_t_next = c->h_dout->t_next;
    c->dev_n_active = c->h_dout->n_active;
    *t_next = c->dev_t_next;
    *n_active = c->dev_n_active;
    *active = c->h_active;
    return HT_OK;
}

namespace {
// Step 4a-6 for the active set of the last ht_dev_next_block: force over the
// lists (or over all particles: the direct scheme), then the corrector.
int dev_step(ht_ctx* c, double eta, double dt_tree, bool direct) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    if (!direct && !c->have_lists) return fail(HT_ESTATE, "interaction lists not set");
    if (c->dev_n_active < 1) return fail(HT_ESTATE, "ht_dev_next_block not called since the last step");
    if (!(eta > 0.0) || !(dt_tree > 0.0)) return fail(HT_EINVAL, "eta and dt_tree must be positive");
    const int32_t n_act = static_cast<int32_t>(c->dev_n_active);
    c->t_pred = c->dev_t_next;
    c->predicted = true;
    int rc = enqueue_step(c, DevRows{}, c->cfg.predict_mode == HT_PREDICT_EAGER, n_act, c->h_active, c->ds.acc,
                          c->ds.jerk, c->ds.fpot, direct);
    if (rc) return rc;
    const CorrEntry e = corr_entry_of(c, 0, eta, dt_tree);
    rc = launch_correct(c->cfg.precision, c->stream, e, nullptr, 0, n_act);
    if (rc) return rc;
    c->dev_n_active = -1;
    c->predicted = false;   // records changed
    return HT_OK;
}
}  // namespace

int ht_dev_step(ht_ctx* c, double eta, double dt_tree) { return dev_step(c, eta, dt_tree, false); }

int ht_dev_step_direct(ht_ctx* c, double eta, double dt_tree) { return dev_step(c, eta, dt_tree, true); }

constexpr int kLoopGraphSteps = 32;  // device-loop steps per captured graph
// Fixed force grid of the device loops (their launch arguments are captured
// in graphs, so the grid cannot follow the item count): eight work-groups per
// resident slot, grid-stride.  Most steps have fewer items than that, so each
// item gets a work-group of its own and the hardware hands them out as slots
// free up, as for the host-planned launches; work-groups past the item count
// exit at once.  (A grid of one work-group per slot assigns items statically and
// was measured about 20% slower on all-particle steps.)
constexpr int kLoopForceGrid = 8192;
constexpr int kLoopCorrGrid = 256;    // fixed corrector grid of the device loop (grid-stride)

namespace {
// The device planner's arguments for a context: its loop state, scheduler
// results, planner scratch and plan region; the launch-table entry it writes
// is `tab` (its own plan region's, or a slot of a batched loop's table).
PlanArgs plan_args_of(const ht_ctx* c, Entry* tab) {
    PlanArgs pa{};
    pa.loop = c->d_loop;
    pa.dout = c->d_dout;
    pa.qmap = c->d_gk;
    pa.active = c->ds.active;
    pa.pgroup = c->d_pgroup;
    pa.loff = c->d_loff;
    pa.qk = c->d_qk;
    pa.qg = c->d_qg;
    pa.tiles = c->d_tiles;
    char* plan = c->ws + c->L.off_plan;
    pa.tab = tab;
    pa.items = reinterpret_cast<Item*>(plan + align_up(kMaxBatch * sizeof(Entry)));
    pa.rtiles = reinterpret_cast<RTile*>(plan + align_up(kMaxBatch * sizeof(Entry)) +
                                         align_up(static_cast<size_t>(c->L.items_max) * sizeof(Item)));
    pa.items_max = c->L.items_max;
    pa.partial_max = c->L.partial_max;
    pa.gather_cost = c->gather_cost;
    pa.target_items = c->target_items;
    pa.d = c->desc();
    pa.d.active = c->ds.active;
    pa.d.acc = c->ds.acc;
    pa.d.jerk = c->ds.jerk;
    pa.d.pot = c->ds.fpot;
    std::memcpy(pa.first_tile, c->first_tile, sizeof(pa.first_tile));
    return pa;
}

// The device loop's scheduler and corrector entries of a context.
SchedEntry loop_sched_entry(const ht_ctx* c, int32_t first_block) {
    SchedEntry se = sched_entry_of(c, first_block);
    se.out = c->d_dout;
    se.active_host = nullptr;
    se.halt = &c->d_loop->halt;
    return se;
}

CorrEntry loop_corr_entry(const ht_ctx* c, const PlanArgs& pa) {
    CorrEntry ce = corr_entry_of(c, 0, 1.0, 1.0);   // eta and dt_tree come from the loop state
    ce.out = c->d_dout;
    ce.loop = c->d_loop;
    ce.qmap = pa.qmap;
    ce.rtiles = pa.rtiles;
    ce.partial = pa.d.partial;
    return ce;
}

// Capture kLoopGraphSteps device-loop steps into one graph.  Every launch
// argument is fixed for the context's life (the call's parameters sit in the
// loop state in device memory), except the work-plan tuning, on whose change
// the graph is captured again.
int build_loop_graph(ht_ctx* c) {
    if (c->loop_exec) {
        (void)hipGraphExecDestroy(c->loop_exec);
        c->loop_exec = nullptr;
    }
    if (c->loop_graph) {
        (void)hipGraphDestroy(c->loop_graph);
        c->loop_graph = nullptr;
    }
    if (!c->cap_stream) HT_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const SchedEntry se = loop_sched_entry(c, 0);
    const PlanArgs pa = plan_args_of(c, reinterpret_cast<Entry*>(c->ws + c->L.off_plan));
    const CorrEntry ce = loop_corr_entry(c, pa);
    const Entry* d_tab = pa.tab;
    hipStream_t s = c->cap_stream;
    HT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kLoopGraphSteps; ++k) {
        sched_min_kernel<<<se.nb, kWG, 0, s>>>(se, nullptr, 0);
        sched_count_kernel<<<se.nb, kWG, 0, s>>>(se, nullptr, 0);
        sched_write_kernel<<<se.nb, kWG, 0, s>>>(se, nullptr, 0);
        dev_plan_kernel<<<1, kPlanWG, 0, s>>>(pa);   // takes the step (or stops the loop) and plans it
        if (c->cfg.precision == HT_PREC_FP64) {
            force_kernel<PrecFp64, false, false><<<kLoopForceGrid, kWG, 0, s>>>(d_tab, 1, -1, &d_tab->n_items);
            dev_correct_kernel<PrecFp64><<<kLoopCorrGrid, kWG, 0, s>>>(ce, nullptr, 0, -1, nullptr);   // sums the splits too
        } else {
            force_kernel<PrecMixed, false, false><<<kLoopForceGrid, kWG, 0, s>>>(d_tab, 1, -1, &d_tab->n_items);
            dev_correct_kernel<PrecMixed><<<kLoopCorrGrid, kWG, 0, s>>>(ce, nullptr, 0, -1, nullptr);
        }
    }
    const hipError_t launch = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(s, &g);
    if (launch != hipSuccess || end != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(HT_EHIP, "capturing the device-loop graph failed: %s",
                    hipGetErrorString(launch != hipSuccess ? launch : end));
    }
    c->loop_graph = g;
    HT_HIP(hipGraphInstantiate(&c->loop_exec, g, nullptr, nullptr, 0));
    c->loop_tuning[0] = c->gather_cost;
    c->loop_tuning[1] = c->target_items;
    c->loop_self_once = c->desc().self_once;
    return HT_OK;
}
}  // namespace


int ht_dev_run(ht_ctx* c, double eta, double dt_tree, double t_stop, int32_t max_steps, int32_t* steps,
               double* t_last, int64_t* particle_steps) {
    if (!c || !steps || !t_last || !particle_steps) return fail(HT_EINVAL, "NULL argument");
    if (!c->ds_mem) return fail(HT_ESTATE, "device state not enabled");
    if (!c->have_lists) return fail(HT_ESTATE, "interaction lists not set");
    if (c->cfg.predict_mode != HT_PREDICT_FUSED) return fail(HT_EINVAL, "the device loop needs fused prediction");
    if (c->list_form != HT_LISTS_CSR) return fail(HT_EINVAL, "the device loop plans CSR lists");
    if (c->gather_cost != std::floor(c->gather_cost))
        return fail(HT_EINVAL, "the device loop plans with a whole-number gather cost (ht_set_tuning)");
    if (!(eta > 0.0) || !(dt_tree > 0.0) || !std::isfinite(t_stop)) return fail(HT_EINVAL, "bad eta, dt_tree or t_stop");
    if (max_steps < 1) return fail(HT_EINVAL, "max_steps < 1");
    *steps = 0;
    *t_last = c->dev_t_next;
    *particle_steps = 0;
    c->dev_n_active = -1;
    if (!c->loop_exec || c->loop_tuning[0] != c->gather_cost || c->loop_tuning[1] != c->target_items ||
        c->loop_self_once != c->desc().self_once) {
        int rc = build_loop_graph(c);
        if (rc) return rc;
    }
    c->slots_all_free();
    loop_init_kernel<<<1, 64, 0, c->stream>>>(c->d_loop, c->d_dout, t_stop, max_steps, eta, dt_tree);
    HT_HIP(hipGetLastError());
    for (int32_t k = 0; k < max_steps; k += kLoopGraphSteps) HT_HIP(hipGraphLaunch(c->loop_exec, c->stream));
    DevLoop L{};
    DevOut o{};
    HT_HIP(hipMemcpyAsync(&L, c->d_loop, sizeof L, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipMemcpyAsync(&o, c->d_dout, sizeof o, hipMemcpyDeviceToHost, c->stream));
    HT_HIP(hipStreamSynchronize(c->stream));
    *steps = static_cast<int32_t>(L.steps);
    *particle_steps = L.psteps;
    if (L.steps > 0) {
        *t_last = L.t_cur;
        c->dev_t_next = L.t_cur;
    }
    c->last_pairs = L.pairs;
    c->predicted = false;
    if (o.below_floor) return fail(HT_ERANGE, "a corrected block step fell below 2^-40");
    if (L.err) return fail(HT_ERANGE, "a device work plan exceeded the context's capacity");
    return HT_OK;
}

int ht_get_predicted(ht_ctx* c, int32_t n, const int32_t* idx, double* xp, double* vp) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!c->have_particles) return fail(HT_ESTATE, "particles not set");
    if (!c->predicted) return fail(HT_ESTATE, "ht_predict not called since the last j-memory change");
    if (n < 0 || (n > 0 && (!idx || !xp || !vp))) return fail(HT_EINVAL, "bad arguments");
    const int32_t jmax = c->n + c->n_nodes;
    for (int32_t k = 0; k < n; ++k)
        if (idx[k] < 0 || idx[k] >= jmax) return fail(HT_ERANGE, "index %d outside [0, %d)", idx[k], jmax);
    char* st = c->ws + c->L.off_stage;
    int32_t* s_idx = reinterpret_cast<int32_t*>(st);
    double* s_x = reinterpret_cast<double*>(st + align_up(kStageRows * 4));
    double* s_v = s_x + 3 * kStageRows;
    const Desc d = c->desc();
    for (int32_t k0 = 0; k0 < n; k0 += kStageRows) {
        const int32_t cnt = std::min<int32_t>(kStageRows, n - k0);
        HT_HIP(hipMemcpyAsync(s_idx, idx + k0, cnt * 4, hipMemcpyHostToDevice, c->stream));
        const int grid = (cnt + kWG - 1) / kWG;
        if (c->cfg.precision == HT_PREC_FP64)
            predict_some_kernel<PrecFp64><<<grid, kWG, 0, c->stream>>>(d, s_idx, cnt, s_x, s_v);
        else
            predict_some_kernel<PrecMixed><<<grid, kWG, 0, c->stream>>>(d, s_idx, cnt, s_x, s_v);
        HT_HIP(hipGetLastError());
        HT_HIP(hipMemcpyAsync(xp + 3 * static_cast<size_t>(k0), s_x, 3 * static_cast<size_t>(cnt) * 8,
                              hipMemcpyDeviceToHost, c->stream));
        HT_HIP(hipMemcpyAsync(vp + 3 * static_cast<size_t>(k0), s_v, 3 * static_cast<size_t>(cnt) * 8,
                              hipMemcpyDeviceToHost, c->stream));
        HT_HIP(hipStreamSynchronize(c->stream));
    }
    return HT_OK;
}

int ht_force_batch_async(int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_active, const int32_t* const* ids,
                         double* const* d_acc, double* const* d_jerk, double* const* d_pot) {
    if (n_ctx < 1 || n_ctx > kMaxBatch) return fail(HT_EINVAL, "n_ctx = %d outside [1, %d]", n_ctx, kMaxBatch);
    if (!ctxs || !n_active || !ids || !d_acc || !d_jerk || !d_pot) return fail(HT_EINVAL, "NULL argument");
    ht_ctx* c0 = ctxs[0];
    if (!c0) return fail(HT_EINVAL, "ctx 0 is NULL");
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        if (!c) return fail(HT_EINVAL, "ctx %d is NULL", k);
        if (c->cfg.device != c0->cfg.device || c->cfg.precision != c0->cfg.precision ||
            c->cfg.predict_mode != c0->cfg.predict_mode)
            return fail(HT_EINVAL, "ctx %d differs in device, precision or predict mode", k);
        if (c->stream != c0->stream) return fail(HT_EINVAL, "ctx %d does not share the stream of ctx 0", k);
        for (int32_t q = 0; q < k; ++q)
            if (ctxs[q] == c) return fail(HT_EINVAL, "ctx %d appears twice in the batch", k);
        if (c->list_form != HT_LISTS_CSR)
            return fail(HT_EINVAL, "ctx %d does not use CSR lists, which batched calls need", k);
        if (!c->have_particles || !c->have_lists) return fail(HT_ESTATE, "ctx %d: lists not set", k);
        if (!c->predicted) return fail(HT_ESTATE, "ctx %d: not predicted", k);
        int rc = validate_active(c, n_active[k], ids[k]);
        if (rc) return rc;
        if (n_active[k] > 0 && (!d_acc[k] || !d_jerk[k] || !d_pot[k])) return fail(HT_EINVAL, "ctx %d: NULL output", k);
    }
    std::vector<Entry> tab;
    tab.reserve(n_ctx);
    int64_t n_items = 0, n_rtiles = 0, pairs = 0;
    int rc = c0->slot_acquire();
    if (rc) return rc;
    const size_t tab_bytes = static_cast<size_t>(n_ctx) * sizeof(Entry);
    size_t end0 = tab_bytes;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        if (n_active[k] == 0) {
            c->last_pairs = 0;
            c->last_items = 0;
            continue;
        }
        rc = plan(c, n_active[k], ids[k], false);
        if (rc) return rc;
        Entry e{};
        if (c == c0) {
            end0 = pack_plan(c, tab_bytes, n_active[k], ids[k], d_acc[k], d_jerk[k], d_pot[k], e);
        } else {
            rc = c->slot_acquire();
            if (rc) return rc;
            rc = copy_plan(c, pack_plan(c, 0, n_active[k], ids[k], d_acc[k], d_jerk[k], d_pot[k], e));
            if (rc) return rc;
        }
        e.first_item = n_items;
        e.first_rtile = n_rtiles;
        n_items += static_cast<int64_t>(c->items.size());
        n_rtiles += static_cast<int64_t>(c->rtiles.size());
        pairs += c->last_pairs;
        tab.push_back(e);
    }
    if (tab.empty()) return HT_OK;
    tab[0].n_items = n_items;
    tab[0].n_rtiles = n_rtiles;
    std::memcpy(c0->plan_host(), tab.data(), tab.size() * sizeof(Entry));
    rc = launch_prep_any(c0->cfg.precision, c0->stream, c0->plan_host(), c0->ws + c0->L.off_plan, end0, nullptr,
                         DevRows{});
    if (rc) return rc;
    rc = c0->slot_release();
    if (rc) return rc;
    const Entry* d_tab = reinterpret_cast<const Entry*>(c0->ws + c0->L.off_plan);
    const int nt = static_cast<int>(tab.size());
    const bool eager = c0->cfg.predict_mode == HT_PREDICT_EAGER;
    if (c0->cfg.precision == HT_PREC_FP64)
        return launch_force<PrecFp64>(c0->stream, eager, c0->tm, d_tab, nt, n_items, n_rtiles, false, pairs);
    return launch_force<PrecMixed>(c0->stream, eager, c0->tm, d_tab, nt, n_items, n_rtiles, false, pairs);
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// batched engine object
namespace {

size_t batch_plan_bytes(int32_t max_clusters, int64_t max_items, int64_t max_active) {
    static_assert(sizeof(CorrEntry) <= 256 && sizeof(SchedEntry) <= 256, "per-cluster tables fit 256 bytes");
    return align_up(static_cast<size_t>(max_clusters) * sizeof(Entry)) +
           align_up(static_cast<size_t>(max_items) * sizeof(Item)) +
           align_up(static_cast<size_t>(max_items) * sizeof(RTile)) + align_up(static_cast<size_t>(max_active) * 4) +
           static_cast<size_t>(max_clusters) * 4 * 256;   // per-cluster alignment and the resident step's tables
}

size_t batch_rows_bytes(int32_t max_clusters, int64_t max_rows) {
    return align_up(static_cast<size_t>(max_clusters) * sizeof(UpdEntry)) + static_cast<size_t>(max_rows) * sizeof(ht_row);
}

constexpr int kMaxLoopCallSteps = 4096;   // engine steps per ht_batch_dev_run call

// The batched device loop's tables, one entry per context of the batch.
struct LoopRegion {
    size_t sched, plan, corr, tab, lctx, counts, ts, total;
};

LoopRegion loop_region(int32_t max_clusters) {
    LoopRegion r{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t m = static_cast<size_t>(max_clusters);
    r.sched = take(m * sizeof(SchedEntry));
    r.plan = take(m * sizeof(PlanArgs));
    r.corr = take(m * sizeof(CorrEntry));
    r.tab = take(m * sizeof(Entry));
    r.lctx = take(m * sizeof(LoopCtx));
    r.counts = take(sizeof(LoopCounts));
    r.ts = take(static_cast<size_t>(kMaxLoopCallSteps) * 8);
    r.total = o;
    return r;
}

bool batch_args_ok(int32_t max_clusters, int64_t max_items, int64_t max_active, int64_t max_rows) {
    return max_clusters >= 1 && max_clusters <= kMaxBatch && max_items >= 1 && max_active >= 1 && max_rows >= 1 &&
           max_items < (int64_t(1) << 31) && max_active < (int64_t(1) << 31) && max_rows < (int64_t(1) << 31);
}

int ring_init(PinnedRing& r, size_t slot_bytes) {
    r.slot_bytes = align_up(slot_bytes);
    if (hipHostMalloc(reinterpret_cast<void**>(&r.base), PinnedRing::kSlots * r.slot_bytes, hipHostMallocDefault) !=
        hipSuccess)
        return fail(HT_ENOMEM, "hipHostMalloc of %zu bytes failed", PinnedRing::kSlots * r.slot_bytes);
    for (int k = 0; k < PinnedRing::kSlots; ++k)
        if (hipEventCreateWithFlags(&r.ev[k], hipEventDisableTiming) != hipSuccess)
            return fail(HT_EHIP, "hipEventCreate failed");
    return HT_OK;
}

void ring_free(PinnedRing& r) {
    for (hipEvent_t e : r.ev)
        if (e) (void)hipEventDestroy(e);
    if (r.base) (void)hipHostFree(r.base);
    r.base = nullptr;
}

int ring_acquire(PinnedRing& r) {
    if (r.pending[r.slot]) {
        HT_HIP(hipEventSynchronize(r.ev[r.slot]));
        r.pending[r.slot] = false;
    }
    return HT_OK;
}

int ring_release(PinnedRing& r, hipStream_t s) {
    HT_HIP(hipEventRecord(r.ev[r.slot], s));
    r.pending[r.slot] = true;
    r.slot = (r.slot + 1) % PinnedRing::kSlots;
    return HT_OK;
}

void ring_all_free(PinnedRing& r) {
    for (bool& p : r.pending) p = false;
}

int check_member(const ht_batch* b, const ht_ctx* c, int32_t k, ht_ctx* const* ctxs, bool same_stream = true) {
    if (!c) return fail(HT_EINVAL, "ctx %d is NULL", k);
    if (c->cfg.device != b->device) return fail(HT_EINVAL, "ctx %d is on another device", k);
    if (same_stream && c->stream != b->stream) return fail(HT_EINVAL, "ctx %d does not share the batch's stream", k);
    if (c->list_form != HT_LISTS_CSR) return fail(HT_EINVAL, "ctx %d does not use CSR lists, which batched calls need", k);
    if (c->cfg.precision != ctxs[0]->cfg.precision || c->cfg.predict_mode != ctxs[0]->cfg.predict_mode)
        return fail(HT_EINVAL, "ctx %d differs in precision or predict mode", k);
    for (int32_t q = 0; q < k; ++q)
        if (ctxs[q] == c) return fail(HT_EINVAL, "ctx %d appears twice", k);
    return HT_OK;
}

}  // namespace

extern "C" {

int ht_batch_workspace_bytes(int32_t max_clusters, int64_t max_items, int64_t max_active, int64_t max_rows,
                             size_t* bytes) {
    if (!bytes || !batch_args_ok(max_clusters, max_items, max_active, max_rows))
        return fail(HT_EINVAL, "invalid batch capacities");
    // update rows are read by the scatter kernel from pinned host staging:
    // the device workspace holds the work plan only
    *bytes = align_up(batch_plan_bytes(max_clusters, max_items, max_active)) + loop_region(max_clusters).total;
    return HT_OK;
}

int ht_batch_create(ht_batch** out, int32_t device, void* stream, int32_t max_clusters, int64_t max_items,
                    int64_t max_active, int64_t max_rows, void* d_workspace, size_t workspace_bytes) {
    if (!out) return fail(HT_EINVAL, "NULL argument");
    *out = nullptr;
    if (!stream) return fail(HT_EINVAL, "a batch needs the stream its contexts share");
    size_t need = 0;
    int rc = ht_batch_workspace_bytes(max_clusters, max_items, max_active, max_rows, &need);
    if (rc) return rc;
    if (d_workspace && (workspace_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255)))
        return fail(HT_EINVAL, "workspace too small or not 256-byte aligned");
    HT_HIP(hipSetDevice(device));
    ht_batch* b = new ht_batch();
    b->device = device;
    b->stream = static_cast<hipStream_t>(stream);
    b->max_clusters = max_clusters;
    b->max_items = max_items;
    b->max_active = max_active;
    b->max_rows = max_rows;
    b->plan_bytes = align_up(batch_plan_bytes(max_clusters, max_items, max_active));
    b->rows_bytes = align_up(batch_rows_bytes(max_clusters, max_rows));
    auto cleanup = [&](int code) {
        ht_batch_destroy(b);
        return code;
    };
    if (d_workspace) {
        b->ws = static_cast<char*>(d_workspace);
    } else {
        if (hipMalloc(&b->ws, need) != hipSuccess) return cleanup(fail(HT_ENOMEM, "hipMalloc of %zu bytes failed", need));
        b->own_ws = true;
    }
    b->loop_ws = b->ws + b->plan_bytes;
    rc = ring_init(b->plan_ring, b->plan_bytes);
    if (rc) return cleanup(rc);
    rc = ring_init(b->rows_ring, b->rows_bytes);
    if (rc) return cleanup(rc);
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_err), sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(HT_ENOMEM, "hipHostMalloc of the error word failed"));
    *b->h_err = 0;
    b->tab.reserve(max_clusters);
    b->utab.reserve(max_clusters);
    *out = b;
    return HT_OK;
}

int ht_batch_destroy(ht_batch* b) {
    if (!b) return HT_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    ring_free(b->plan_ring);
    ring_free(b->rows_ring);
    if (b->h_err) (void)hipHostFree(b->h_err);
    if (b->loop_exec) (void)hipGraphExecDestroy(b->loop_exec);
    if (b->loop_graph) (void)hipGraphDestroy(b->loop_graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_lparams) (void)hipHostFree(b->h_lparams);
    if (b->h_lres) (void)hipHostFree(b->h_lres);
    if (b->h_ts) (void)hipHostFree(b->h_ts);
    for (hipEvent_t e : b->tm.pool) (void)hipEventDestroy(e);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    delete b;
    return HT_OK;
}

}  // extern "C"

namespace {

// Validate the rows of a batched update and launch the row scatter.  copy:
// the rows are copied into the batch's pinned staging (the caller's arrays may
// be anything and are free on return); otherwise the kernel reads the caller's
// arrays, which must be pinned and stay unchanged until the stream passes.
int batch_update(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_rows, const ht_row* const* rows,
                 bool copy) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (n_ctx < 0 || n_ctx > b->max_clusters) return fail(HT_EINVAL, "n_ctx = %d outside [0, %d]", n_ctx, b->max_clusters);
    if (n_ctx == 0) return HT_OK;
    if (!ctxs || !n_rows || !rows) return fail(HT_EINVAL, "NULL argument");
    int64_t total = 0;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        int rc = check_member(b, c, k, ctxs);
        if (rc) return rc;
        if (!c->have_particles) return fail(HT_ESTATE, "ctx %d: particles not set", k);
        if (n_rows[k] < 0 || (n_rows[k] > 0 && !rows[k])) return fail(HT_EINVAL, "ctx %d: bad rows", k);
        // indices in range and distinct: one sequential pass when they are
        // increasing (the usual case: rows of an ascending active set), else marks
        bool increasing = true;
        for (int32_t r = 0; r < n_rows[k]; ++r) {
            const int32_t j = rows[k][r].idx;
            if (j < 0 || j >= c->n) return fail(HT_ERANGE, "ctx %d: row index %d outside [0, %d)", k, j, c->n);
            if (r > 0 && j <= rows[k][r - 1].idx) increasing = false;
        }
        if (!increasing) {
            if (c->mark.size() != static_cast<size_t>(c->n)) c->mark.assign(static_cast<size_t>(c->n), 0u);
            if (++c->mark_gen == 0) {
                std::fill(c->mark.begin(), c->mark.end(), 0u);
                c->mark_gen = 1;
            }
            for (int32_t r = 0; r < n_rows[k]; ++r) {
                const int32_t j = rows[k][r].idx;
                if (c->mark[j] == c->mark_gen) return fail(HT_EINVAL, "ctx %d: particle %d updated twice", k, j);
                c->mark[j] = c->mark_gen;
            }
        }
        total += n_rows[k];
    }
    if (total > b->max_rows) return fail(HT_ERANGE, "%lld update rows over capacity %lld", (long long)total,
                                         (long long)b->max_rows);
    for (int32_t k = 0; k < n_ctx; ++k) ctxs[k]->predicted = false;
    if (total == 0) return HT_OK;
    int rc = ring_acquire(b->rows_ring);
    if (rc) return rc;
    char* hs = b->rows_ring.host();
    b->utab.clear();
    int64_t first = 0;
    const size_t rows_at = align_up(static_cast<size_t>(n_ctx) * sizeof(UpdEntry));
    for (int32_t k = 0; k < n_ctx; ++k) {
        if (n_rows[k] == 0) continue;
        const ht_row* src = rows[k];
        if (copy) {
            ht_row* dst = reinterpret_cast<ht_row*>(hs + rows_at) + first;
            std::memcpy(dst, rows[k], static_cast<size_t>(n_rows[k]) * sizeof(ht_row));
            src = dst;
        }
        b->utab.push_back(UpdEntry{ctxs[k]->ws + ctxs[k]->L.off_rec, first, src, ctxs[k]->n});
        first += n_rows[k];
    }
    std::memcpy(hs, b->utab.data(), b->utab.size() * sizeof(UpdEntry));
    const int grid = static_cast<int>(std::min<int64_t>((total + kWG - 1) / kWG, 65536));
    const UpdEntry* h_tab = reinterpret_cast<const UpdEntry*>(hs);
    const int nt = static_cast<int>(b->utab.size());
    if (ctxs[0]->cfg.precision == HT_PREC_FP64)
        scatter_rows_kernel<PrecFp64><<<grid, kWG, 0, b->stream>>>(h_tab, nt, total, b->h_err);
    else
        scatter_rows_kernel<PrecMixed><<<grid, kWG, 0, b->stream>>>(h_tab, nt, total, b->h_err);
    HT_HIP(hipGetLastError());
    return ring_release(b->rows_ring, b->stream);   // the kernel is the slot's last reader
}

}  // namespace

extern "C" {

int ht_batch_update_async(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_rows,
                          const ht_row* const* rows) {
    return batch_update(b, n_ctx, ctxs, n_rows, rows, true);
}

int ht_batch_update_pinned_async(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_rows,
                                 const ht_row* const* rows) {
    return batch_update(b, n_ctx, ctxs, n_rows, rows, false);
}

}  // extern "C"

namespace {

// The batched force launch; `extra` (extra_bytes) is appended to the packed
// plan and reaches the device with it, at *extra_dev.
// own_lists: the active lists are the contexts' own scheduler results (ascending
// and in range by construction), so only their sizes are checked, as dev_step does.
int batch_force(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_active, const int32_t* const* ids,
                double* const* d_acc, double* const* d_jerk, double* const* d_pot, const void* extra,
                size_t extra_bytes, char** extra_dev, bool own_lists = false) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (n_ctx < 0 || n_ctx > b->max_clusters) return fail(HT_EINVAL, "n_ctx = %d outside [0, %d]", n_ctx, b->max_clusters);
    b->last_pairs = 0;
    b->last_items = 0;
    if (n_ctx == 0) return HT_OK;
    if (!ctxs || !n_active || !ids || !d_acc || !d_jerk || !d_pot) return fail(HT_EINVAL, "NULL argument");
    int64_t act_total = 0;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        int rc = check_member(b, c, k, ctxs);
        if (rc) return rc;
        if (!c->have_particles || !c->have_lists) return fail(HT_ESTATE, "ctx %d: lists not set", k);
        if (!c->predicted) return fail(HT_ESTATE, "ctx %d: not predicted", k);
        if (own_lists) {
            if (n_active[k] < 0 || n_active[k] > c->cfg.active_max || (n_active[k] > 0 && !ids[k]))
                return fail(HT_ERANGE, "ctx %d: active list of %d outside the capacity %d", k, n_active[k],
                            c->cfg.active_max);
        } else {
            rc = validate_active(c, n_active[k], ids[k]);
            if (rc) return rc;
        }
        if (n_active[k] > 0 && (!d_acc[k] || !d_jerk[k] || !d_pot[k])) return fail(HT_EINVAL, "ctx %d: NULL output", k);
        act_total += n_active[k];
    }
    if (act_total > b->max_active) return fail(HT_ERANGE, "%lld active particles over the batch capacity %lld",
                                               (long long)act_total, (long long)b->max_active);
    int rc = ring_acquire(b->plan_ring);
    if (rc) return rc;
    char* hs = b->plan_ring.host();
    char* dv = b->ws;
    b->tab.clear();
    int64_t n_items = 0, n_rtiles = 0, pairs = 0;
    size_t at = static_cast<size_t>(n_ctx) * sizeof(Entry);
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        if (n_active[k] == 0) {
            c->last_pairs = 0;
            c->last_items = 0;
            continue;
        }
        rc = plan(c, n_active[k], ids[k], false);
        if (rc) return rc;
        if (n_items + static_cast<int64_t>(c->items.size()) > b->max_items ||
            n_rtiles + static_cast<int64_t>(c->rtiles.size()) > b->max_items)
            return fail(HT_ERANGE, "work items over the batch capacity %lld", (long long)b->max_items);
        Entry e{};
        at = pack_plan_into(c, hs, dv, at, n_active[k], ids[k], d_acc[k], d_jerk[k], d_pot[k], e);
        e.first_item = n_items;
        e.first_rtile = n_rtiles;
        n_items += static_cast<int64_t>(c->items.size());
        n_rtiles += static_cast<int64_t>(c->rtiles.size());
        pairs += c->last_pairs;
        b->tab.push_back(e);
    }
    if (b->tab.empty()) return HT_OK;
    if (extra_bytes) {
        at = align_up(at);
        if (at + extra_bytes <= b->plan_bytes) std::memcpy(hs + at, extra, extra_bytes);
        *extra_dev = dv + at;
        at += extra_bytes;
    }
    if (at > b->plan_bytes) return fail(HT_ERANGE, "batch plan over its capacity");
    b->tab[0].n_items = n_items;
    b->tab[0].n_rtiles = n_rtiles;
    std::memcpy(hs, b->tab.data(), b->tab.size() * sizeof(Entry));
    rc = launch_prep_any(ctxs[0]->cfg.precision, b->stream, hs, dv, at, nullptr, DevRows{});
    if (rc) return rc;
    rc = ring_release(b->plan_ring, b->stream);
    if (rc) return rc;
    b->last_pairs = pairs;
    b->last_items = static_cast<int32_t>(n_items);
    const Entry* d_tab = reinterpret_cast<const Entry*>(dv);
    const int nt = static_cast<int>(b->tab.size());
    const bool eager = ctxs[0]->cfg.predict_mode == HT_PREDICT_EAGER;
    if (ctxs[0]->cfg.precision == HT_PREC_FP64)
        return launch_force<PrecFp64>(b->stream, eager, b->tm, d_tab, nt, n_items, n_rtiles, false, pairs);
    return launch_force<PrecMixed>(b->stream, eager, b->tm, d_tab, nt, n_items, n_rtiles, false, pairs);
}

}  // namespace

extern "C" {

int ht_batch_force_async(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const int32_t* n_active,
                         const int32_t* const* ids, double* const* d_acc, double* const* d_jerk, double* const* d_pot) {
    return batch_force(b, n_ctx, ctxs, n_active, ids, d_acc, d_jerk, d_pot, nullptr, 0, nullptr);
}

// ------------------------------------------------------------------------------------------------
// device-resident batched steps
int ht_batch_dev_next_block(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, double* t_next, int64_t* n_active,
                            const int32_t** active) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (n_ctx < 1 || n_ctx > b->max_clusters) return fail(HT_EINVAL, "n_ctx = %d outside [1, %d]", n_ctx, b->max_clusters);
    if (!ctxs || !t_next || !n_active || !active) return fail(HT_EINVAL, "NULL argument");
    std::vector<SchedEntry> tab;
    tab.reserve(n_ctx);
    int32_t blocks = 0;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        int rc = check_member(b, c, k, ctxs);
        if (rc) return rc;
        if (!c->ds_mem) return fail(HT_ESTATE, "ctx %d: device state not enabled", k);
        if (c->n < 1) return fail(HT_ESTATE, "ctx %d: particles not set", k);
        tab.push_back(sched_entry_of(c, blocks));
        blocks += tab.back().nb;
    }
    int rc = ring_acquire(b->plan_ring);
    if (rc) return rc;
    const size_t bytes = tab.size() * sizeof(SchedEntry);
    std::memcpy(b->plan_ring.host(), tab.data(), bytes);
    rc = launch_prep_any(ctxs[0]->cfg.precision, b->stream, b->plan_ring.host(), b->ws, bytes, nullptr, DevRows{});
    if (rc) return rc;
    rc = ring_release(b->plan_ring, b->stream);
    if (rc) return rc;
    const SchedEntry* d_tab = reinterpret_cast<const SchedEntry*>(b->ws);
    const SchedEntry none{};
    sched_min_kernel<<<blocks, kWG, 0, b->stream>>>(none, d_tab, n_ctx);
    sched_count_kernel<<<blocks, kWG, 0, b->stream>>>(none, d_tab, n_ctx);
    sched_write_kernel<<<blocks, kWG, 0, b->stream>>>(none, d_tab, n_ctx);
    HT_HIP(hipGetLastError());
    HT_HIP(hipStreamSynchronize(b->stream));
    ring_all_free(b->plan_ring);
    ring_all_free(b->rows_ring);
    int bad = -1;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        c->slots_all_free();
        if (c->h_dout->below_floor) {
            c->h_dout->below_floor = 0;
            if (bad < 0) bad = k;
        }
        c->dev_t_next = c->h_dout->t_next;
        c->dev_n_active = c->h_dout->n_active;
        t_next[k] = c->dev_t_next;
        n_active[k] = c->dev_n_active;
        active[k] = c->h_active;
    }
    if (bad >= 0) return fail(HT_ERANGE, "ctx %d: a corrected block step fell below 2^-40", bad);
    return take_row_error(b->h_err);
}

int ht_batch_dev_step(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const double* eta, const double* dt_tree) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (n_ctx < 1 || n_ctx > b->max_clusters) return fail(HT_EINVAL, "n_ctx = %d outside [1, %d]", n_ctx, b->max_clusters);
    if (!ctxs || !eta || !dt_tree) return fail(HT_EINVAL, "NULL argument");
    std::vector<int32_t> n_act(n_ctx);
    std::vector<const int32_t*> ids(n_ctx);
    std::vector<double*> acc(n_ctx), jerk(n_ctx), pot(n_ctx);
    std::vector<CorrEntry> corr(n_ctx);
    int64_t rows = 0;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        if (!c || !c->ds_mem) return fail(HT_ESTATE, "ctx %d: device state not enabled", k);
        if (c->dev_n_active < 1) return fail(HT_ESTATE, "ctx %d: no next block since the last step", k);
        if (!(eta[k] > 0.0) || !(dt_tree[k] > 0.0)) return fail(HT_EINVAL, "ctx %d: eta and dt_tree must be positive", k);
        c->t_pred = c->dev_t_next;
        c->predicted = true;
        n_act[k] = static_cast<int32_t>(c->dev_n_active);
        ids[k] = c->h_active;
        acc[k] = c->ds.acc;
        jerk[k] = c->ds.jerk;
        pot[k] = c->ds.fpot;
        corr[k] = corr_entry_of(c, rows, eta[k], dt_tree[k]);
        rows += n_act[k];
    }
    char* d_corr = nullptr;
    int rc = batch_force(b, n_ctx, ctxs, n_act.data(), ids.data(), acc.data(), jerk.data(), pot.data(), corr.data(),
                         corr.size() * sizeof(CorrEntry), &d_corr, true);
    if (rc) return rc;
    rc = launch_correct(ctxs[0]->cfg.precision, b->stream, corr[0], reinterpret_cast<const CorrEntry*>(d_corr), n_ctx,
                        rows);
    if (rc) return rc;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ctxs[k]->dev_n_active = -1;
        ctxs[k]->predicted = false;
    }
    return HT_OK;
}

}  // extern "C"

namespace {

// Capture kLoopGraphSteps engine steps of the batched device loop over the
// n_ctx contexts whose tables sit in the batch's loop region.
template <class P>
int build_batch_loop_graph(ht_batch* b, int32_t n_ctx) {
    if (b->loop_exec) {
        (void)hipGraphExecDestroy(b->loop_exec);
        b->loop_exec = nullptr;
    }
    if (b->loop_graph) {
        (void)hipGraphDestroy(b->loop_graph);
        b->loop_graph = nullptr;
    }
    if (!b->cap_stream) HT_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    const LoopRegion R = loop_region(b->max_clusters);
    char* w = b->loop_ws;
    const SchedEntry* d_sched = reinterpret_cast<const SchedEntry*>(w + R.sched);
    const PlanArgs* d_plan = reinterpret_cast<const PlanArgs*>(w + R.plan);
    CorrEntry* d_corr = reinterpret_cast<CorrEntry*>(w + R.corr);
    Entry* d_tab = reinterpret_cast<Entry*>(w + R.tab);
    const LoopCtx* d_lctx = reinterpret_cast<const LoopCtx*>(w + R.lctx);
    LoopCounts* d_cnt = reinterpret_cast<LoopCounts*>(w + R.counts);
    int64_t* d_ts = reinterpret_cast<int64_t*>(w + R.ts);
    const SchedEntry none{};
    const CorrEntry cnone{};
    hipStream_t s = b->cap_stream;
    HT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kLoopGraphSteps; ++k) {
        sched_min_kernel<<<b->loop_blocks, kWG, 0, s>>>(none, d_sched, n_ctx);
        sched_count_kernel<<<b->loop_blocks, kWG, 0, s>>>(none, d_sched, n_ctx);
        sched_write_kernel<<<b->loop_blocks, kWG, 0, s>>>(none, d_sched, n_ctx);
        dev_plan_batch_kernel<<<n_ctx, kPlanWG, 0, s>>>(d_plan);   // each context takes its step (or stops) and plans it
        batch_loop_table_kernel<<<1, kLoopTabWG, 0, s>>>(d_tab, d_corr, d_lctx, n_ctx, d_cnt, d_ts, kMaxLoopCallSteps);
        force_kernel<P, false, false><<<kLoopForceGrid, kWG, 0, s>>>(d_tab, n_ctx, -1, &d_cnt->items);
        dev_correct_kernel<P><<<kLoopCorrGrid, kWG, 0, s>>>(cnone, d_corr, n_ctx, -1, &d_cnt->rows);
    }
    const hipError_t launch = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(s, &g);
    if (launch != hipSuccess || end != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(HT_EHIP, "capturing the batched device-loop graph failed: %s",
                    hipGetErrorString(launch != hipSuccess ? launch : end));
    }
    b->loop_graph = g;
    HT_HIP(hipGraphInstantiate(&b->loop_exec, g, nullptr, nullptr, 0));
    return HT_OK;
}

// The tables of the batched device loop for these contexts, and its graph,
// unless the last call used the same contexts with the same sizes and tunings.
int prepare_batch_loop(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs) {
    std::vector<double> key;
    key.reserve(static_cast<size_t>(n_ctx) * 3);
    for (int32_t k = 0; k < n_ctx; ++k) {
        key.push_back(static_cast<double>(ctxs[k]->n));
        key.push_back(ctxs[k]->gather_cost);
        key.push_back(ctxs[k]->target_items);
        key.push_back(static_cast<double>(ctxs[k]->desc().self_once));
    }
    if (b->loop_exec && b->loop_ctxs.size() == static_cast<size_t>(n_ctx) &&
        std::equal(b->loop_ctxs.begin(), b->loop_ctxs.end(), ctxs) && b->loop_key == key)
        return HT_OK;
    const LoopRegion R = loop_region(b->max_clusters);
    char* w = b->loop_ws;
    std::vector<SchedEntry> sched(n_ctx);
    std::vector<PlanArgs> plan(n_ctx);
    std::vector<CorrEntry> corr(n_ctx);
    std::vector<LoopCtx> lctx(n_ctx);
    std::vector<Entry> tab(n_ctx);
    int32_t blocks = 0;
    for (int32_t k = 0; k < n_ctx; ++k) {
        const ht_ctx* c = ctxs[k];
        sched[k] = loop_sched_entry(c, blocks);
        blocks += sched[k].nb;
        plan[k] = plan_args_of(c, reinterpret_cast<Entry*>(w + R.tab) + k);
        corr[k] = loop_corr_entry(c, plan[k]);
        lctx[k] = LoopCtx{c->d_loop, c->d_dout};
        tab[k] = Entry{};
    }
    const size_t nk = static_cast<size_t>(n_ctx);
    HT_HIP(hipMemcpyAsync(w + R.sched, sched.data(), nk * sizeof(SchedEntry), hipMemcpyHostToDevice, b->stream));
    HT_HIP(hipMemcpyAsync(w + R.plan, plan.data(), nk * sizeof(PlanArgs), hipMemcpyHostToDevice, b->stream));
    HT_HIP(hipMemcpyAsync(w + R.corr, corr.data(), nk * sizeof(CorrEntry), hipMemcpyHostToDevice, b->stream));
    HT_HIP(hipMemcpyAsync(w + R.lctx, lctx.data(), nk * sizeof(LoopCtx), hipMemcpyHostToDevice, b->stream));
    HT_HIP(hipMemcpyAsync(w + R.tab, tab.data(), nk * sizeof(Entry), hipMemcpyHostToDevice, b->stream));
    HT_HIP(hipStreamSynchronize(b->stream));   // pageable sources
    b->loop_blocks = blocks;
    const int rc = ctxs[0]->cfg.precision == HT_PREC_FP64 ? build_batch_loop_graph<PrecFp64>(b, n_ctx)
                                                           : build_batch_loop_graph<PrecMixed>(b, n_ctx);
    if (rc) {
        b->loop_ctxs.clear();
        return rc;
    }
    b->loop_ctxs.assign(ctxs, ctxs + n_ctx);
    b->loop_key = key;
    return HT_OK;
}

}  // namespace

extern "C" {

int ht_batch_dev_run(ht_batch* b, int32_t n_ctx, ht_ctx* const* ctxs, const double* eta, const double* dt_tree,
                     const double* t_stop, const int32_t* max_steps, int32_t engine_steps, int32_t* steps,
                     double* t_last, int64_t* particle_steps, int64_t* pairs, double* step_ms,
                     int32_t* n_step_ms) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (n_ctx < 1 || n_ctx > b->max_clusters) return fail(HT_EINVAL, "n_ctx = %d outside [1, %d]", n_ctx, b->max_clusters);
    if (!ctxs || !eta || !dt_tree || !t_stop || !max_steps || !steps || !t_last || !particle_steps || !pairs ||
        !step_ms || !n_step_ms)
        return fail(HT_EINVAL, "NULL argument");
    if (engine_steps < 1 || engine_steps > kMaxLoopCallSteps)
        return fail(HT_EINVAL, "engine_steps = %d outside [1, %d]", engine_steps, kMaxLoopCallSteps);
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        int rc = check_member(b, c, k, ctxs, false);
        if (rc) return rc;
        if (max_steps[k] < 0) return fail(HT_EINVAL, "ctx %d: max_steps < 0", k);
        if (max_steps[k] == 0) continue;   // sits out: its host state may be in use elsewhere
        if (!c->ds_mem) return fail(HT_ESTATE, "ctx %d: device state not enabled", k);
        if (!c->have_lists) return fail(HT_ESTATE, "ctx %d: interaction lists not set", k);
        if (c->cfg.predict_mode != HT_PREDICT_FUSED) return fail(HT_EINVAL, "ctx %d: the device loop needs fused prediction", k);
        if (c->gather_cost != std::floor(c->gather_cost))
            return fail(HT_EINVAL, "ctx %d: the device loop plans with a whole-number gather cost", k);
        if (!(eta[k] > 0.0) || !(dt_tree[k] > 0.0) || !std::isfinite(t_stop[k]))
            return fail(HT_EINVAL, "ctx %d: bad eta, dt_tree or t_stop", k);
    }
    int rc = prepare_batch_loop(b, n_ctx, ctxs);
    if (rc) return rc;
    if (!b->h_lparams) {
        const size_t m = static_cast<size_t>(b->max_clusters);
        if (hipHostMalloc(reinterpret_cast<void**>(&b->h_lparams), m * sizeof(LoopParams), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&b->h_lres), m * sizeof(LoopResult), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&b->h_ts), (kMaxLoopCallSteps + 2) * sizeof(int64_t),
                          hipHostMallocDefault) != hipSuccess)
            return fail(HT_ENOMEM, "hipHostMalloc for the batched device loop failed");
    }
    for (int32_t k = 0; k < n_ctx; ++k) {
        b->h_lparams[k] = LoopParams{t_stop[k], eta[k], dt_tree[k], std::min<int64_t>(max_steps[k], engine_steps)};
        if (max_steps[k] == 0) continue;
        ctxs[k]->dev_n_active = -1;
        ctxs[k]->slots_all_free();
    }
    const LoopRegion R = loop_region(b->max_clusters);
    char* w = b->loop_ws;
    const LoopCtx* d_lctx = reinterpret_cast<const LoopCtx*>(w + R.lctx);
    LoopCounts* d_cnt = reinterpret_cast<LoopCounts*>(w + R.counts);
    const int64_t* d_ts = reinterpret_cast<const int64_t*>(w + R.ts);
    const int grid = (n_ctx + kWG - 1) / kWG;
    batch_loop_init_kernel<<<grid, kWG, 0, b->stream>>>(d_lctx, b->h_lparams, n_ctx, d_cnt);
    HT_HIP(hipGetLastError());
    for (int32_t q = 0; q < engine_steps; q += kLoopGraphSteps) HT_HIP(hipGraphLaunch(b->loop_exec, b->stream));
    batch_loop_results_kernel<<<grid, kWG, 0, b->stream>>>(d_lctx, n_ctx, b->h_lres, d_cnt, d_ts, kMaxLoopCallSteps,
                                                          b->h_ts);
    HT_HIP(hipGetLastError());
    HT_HIP(hipStreamSynchronize(b->stream));
    ring_all_free(b->plan_ring);
    ring_all_free(b->rows_ring);
    int bad = -1, bad_plan = -1;
    for (int32_t k = 0; k < n_ctx; ++k) {
        ht_ctx* c = ctxs[k];
        const LoopResult& r = b->h_lres[k];
        steps[k] = static_cast<int32_t>(r.steps);
        particle_steps[k] = r.psteps;
        pairs[k] = r.pairs;
        if (max_steps[k] == 0) {
            t_last[k] = std::numeric_limits<double>::quiet_NaN();
            continue;
        }
        if (r.steps > 0) c->dev_t_next = r.t_cur;
        t_last[k] = c->dev_t_next;
        c->last_pairs = r.pairs;
        c->predicted = false;
        if (r.below_floor && bad < 0) bad = k;
        if (r.err && bad_plan < 0) bad_plan = k;
    }
    int rate_khz = 0;
    HT_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device));
    const int64_t m = std::min<int64_t>(b->h_ts[0], engine_steps);
    for (int64_t q = 0; q < m; ++q)
        step_ms[q] = static_cast<double>(b->h_ts[2 + q] - b->h_ts[1 + q]) / std::max(rate_khz, 1);
    *n_step_ms = static_cast<int32_t>(m);
    if (bad >= 0) return fail(HT_ERANGE, "ctx %d: a corrected block step fell below 2^-40", bad);
    if (bad_plan >= 0) return fail(HT_ERANGE, "ctx %d: a device work plan exceeded the context's capacity", bad_plan);
    return take_row_error(b->h_err);
}

int ht_batch_sync(ht_batch* b) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    HT_HIP(hipStreamSynchronize(b->stream));
    ring_all_free(b->plan_ring);
    ring_all_free(b->rows_ring);
    if (int rc = take_row_error(b->h_err)) return rc;
    return HT_OK;
}

int ht_batch_set_timing(ht_batch* b, int32_t enable) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    b->tm.enabled = enable != 0;
    b->tm.used = 0;
    b->tm.pairs = 0;
    return HT_OK;
}

int ht_batch_kernel_timing(ht_batch* b, double* force_ms, int64_t* launches, int64_t* pairs) {
    if (!b || !force_ms || !launches || !pairs) return fail(HT_EINVAL, "NULL argument");
    int rc = read_timing(b->stream, b->tm, force_ms, launches, pairs);
    if (rc == HT_OK) {
        ring_all_free(b->plan_ring);
        ring_all_free(b->rows_ring);
    }
    return rc;
}

int ht_batch_last_stats(const ht_batch* b, int64_t* pairs, int32_t* work_items) {
    if (!b) return fail(HT_EINVAL, "batch is NULL");
    if (pairs) *pairs = b->last_pairs;
    if (work_items) *work_items = b->last_items;
    return HT_OK;
}

}  // extern "C"

extern "C" {

int ht_sync(ht_ctx* c) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    return ctx_sync(c);
}

int ht_set_timing(ht_ctx* c, int32_t enable) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    c->tm.enabled = enable != 0;
    c->tm.used = 0;
    c->tm.pairs = 0;
    return HT_OK;
}

int ht_kernel_timing(ht_ctx* c, double* force_ms, int64_t* launches, int64_t* pairs) {
    if (!c || !force_ms || !launches || !pairs) return fail(HT_EINVAL, "NULL argument");
    int rc = read_timing(c->stream, c->tm, force_ms, launches, pairs);
    if (rc == HT_OK) {
        c->slots_all_free();
        rc = take_row_error(c->h_err);
    }
    return rc;
}

int ht_set_tuning(ht_ctx* c, double gather_cost, double target_items) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (!(gather_cost >= 0.0 && gather_cost < 1e6) || !(target_items >= 1.0 && target_items < 1e8))
        return fail(HT_EINVAL, "tuning values out of range");
    c->gather_cost = gather_cost;
    c->target_items = target_items;
    tile_table(gather_cost, c->first_tile);
    return HT_OK;
}

int ht_set_placement(ht_ctx* c, int32_t runs) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (runs < 0 || runs > kMaxBins) return fail(HT_EINVAL, "placement runs = %d outside [0, %d]", runs, kMaxBins);
    c->placement = runs == 0 ? c->n_xcc : runs;
    return HT_OK;
}

int ht_get_placement(const ht_ctx* c, int32_t* runs, int32_t* n_xcc) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (runs) *runs = c->placement;
    if (n_xcc) *n_xcc = c->n_xcc;
    return HT_OK;
}

int ht_last_stats(const ht_ctx* c, int64_t* pairs, int32_t* work_items) {
    if (!c) return fail(HT_EINVAL, "ctx is NULL");
    if (pairs) *pairs = c->last_pairs;
    if (work_items) *work_items = c->last_items;
    return HT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Admission by device footprint (the served stream): a pool is a budget of
// device bytes on one GPU and the reservations held against it.  It
// allocates nothing; a cluster's reservation is what its context and (when
// resident) its device state will hold, from the same layouts ht_create and
// ht_state_enable use.
struct ht_pool {
    int32_t device = 0;
    size_t budget = 0, used = 0;
    int64_t next_id = 1;
    std::vector<std::pair<int64_t, size_t>> held;   // (id, bytes)
    std::mutex mu;
};

namespace {
int pool_take(ht_pool* p, size_t bytes, int64_t* id) {
    std::lock_guard<std::mutex> lock(p->mu);
    if (bytes > p->budget)
        return fail(HT_ERANGE, "%zu bytes exceed the whole budget of %zu bytes", bytes, p->budget);
    if (p->used + bytes > p->budget)
        return fail(HT_ENOMEM, "%zu bytes do not fit: %zu of %zu bytes held", bytes, p->used, p->budget);
    *id = p->next_id++;
    p->held.emplace_back(*id, bytes);
    p->used += bytes;
    return HT_OK;
}
}  // namespace

extern "C" {

int ht_pool_create(ht_pool** out, int32_t device, size_t budget_bytes) {
    if (!out) return fail(HT_EINVAL, "NULL argument");
    *out = nullptr;
    if (device < 0) return fail(HT_EINVAL, "device %d < 0", device);
    ht_pool* p = new ht_pool();
    p->device = device;
    p->budget = budget_bytes;
    *out = p;
    return HT_OK;
}

int ht_pool_destroy(ht_pool* p) {
    delete p;
    return HT_OK;
}


int ht_cluster_admit(ht_pool* p, const ht_config* cfg, int32_t resident, int64_t* id, size_t* bytes) {
    if (!p || !cfg || !id) return fail(HT_EINVAL, "NULL argument");
    Layout L;
    if (!layout_of(*cfg, L)) return fail(HT_EINVAL, "invalid configuration");
    if (cfg->device != p->device) return fail(HT_EINVAL, "configuration for device %d, pool on %d", cfg->device, p->device);
    const size_t need = L.total + (resident ? state_layout(*cfg).total : 0);
    if (bytes) *bytes = need;
    return pool_take(p, need, id);
}

int ht_pool_reserve(ht_pool* p, size_t bytes, int64_t* id) {
    if (!p || !id) return fail(HT_EINVAL, "NULL argument");
    return pool_take(p, bytes, id);
}

int ht_pool_resize(ht_pool* p, int64_t id, size_t bytes) {
    if (!p) return fail(HT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto& h : p->held)
        if (h.first == id) {
            p->used = p->used - h.second + bytes;
            h.second = bytes;
            if (p->used > p->budget)
                return fail(HT_ENOMEM, "reservation %lld now holds %zu bytes: %zu of %zu bytes held", (long long)id,
                            bytes, p->used, p->budget);
            return HT_OK;
        }
    return fail(HT_EINVAL, "no reservation %lld", (long long)id);
}

int ht_cluster_release(ht_pool* p, int64_t id) {
    if (!p) return fail(HT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    for (size_t k = 0; k < p->held.size(); ++k)
        if (p->held[k].first == id) {
            p->used -= p->held[k].second;
            p->held.erase(p->held.begin() + static_cast<std::ptrdiff_t>(k));
            return HT_OK;
        }
    return fail(HT_EINVAL, "no reservation %lld", (long long)id);
}

int ht_pool_usage(ht_pool* p, size_t* used, size_t* budget, int32_t* n_held) {
    if (!p) return fail(HT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    if (used) *used = p->used;
    if (budget) *budget = p->budget;
    if (n_held) *n_held = static_cast<int32_t>(p->held.size());
    return HT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Direct sum with no allocation (ht_force_direct_noalloc): the force of the
// original Hermite scheme (Section 2) on caller-owned device arrays of
// predicted positions, velocities and masses.  The j-range is cut into
// j_splits ranges summed by separate work-groups; their partial sums live in
// `scratch`, one fixed array per device that the library holds until the
// process ends, and a second kernel adds them in split order.  Nothing in it
// must start at zero: every partial slot a call reads was written by that
// call's first kernel.
constexpr size_t kScratchBytes = HT_NOALLOC_SCRATCH_BYTES;   // per device

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// The device address of `scratch` on `device` (taken once per device, with
// that device current; the array's name in host code is not that address).
int scratch_on(int32_t device, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int prev = 0;
        HT_HIP(hipGetDevice(&prev));
        HT_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t back = hipSetDevice(prev);
        if (e != hipSuccess) return fail(HT_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (back != hipSuccess) return fail(HT_EHIP, "hipSetDevice: %s", hipGetErrorString(back));
        g_scratch[device] = static_cast<double*>(p);
    }
    *out = g_scratch[device];
    return HT_OK;
}

// Work-group (tile, split): 256 active particles of one tile against the
// split's j-range, staged through LDS 256 entries at a time; the same pair
// arithmetic as the list force.  An active id outside [0, n) gives NaN in its
// output row (the ids sit in device memory, so the host cannot check them).
template <class P>
__global__ __launch_bounds__(kWG) void noalloc_direct_kernel(int32_t n, const double* __restrict__ x,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ m, double eps2,
                                                             int32_t n_active, const int32_t* __restrict__ active,
                                                             int64_t per, double* part, double* acc, double* jerk,
                                                             double* pot) {
    using V = typename P::Vel;
    using S = typename P::Stored;
    __shared__ JRec<P> tile[kWG];
    const int tid = threadIdx.x;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kWG + tid;
    const int split = blockIdx.y;
    const bool has_q = q < n_active;
    const int32_t i_raw = has_q ? active[q] : 0;
    const bool ok = i_raw >= 0 && i_raw < n;
    const int32_t i = ok ? i_raw : 0;
    const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
    const V vxi = static_cast<V>(v[3 * i]), vyi = static_cast<V>(v[3 * i + 1]), vzi = static_cast<V>(v[3 * i + 2]);
    Acc64 A;
#pragma unroll
    for (int k = 0; k < kOut; ++k) A.v[k] = 0.0;
    const int64_t jb = split * per, je = jb + per < n ? jb + per : n;
    for (int64_t base = jb; base < je; base += kWG) {
        const int cnt = je - base < kWG ? static_cast<int>(je - base) : kWG;
        __syncthreads();
        if (tid < cnt) {
            const int64_t j = base + tid;
            tile[tid] = JRec<P>{x[3 * j], x[3 * j + 1], x[3 * j + 2], static_cast<V>(v[3 * j]),
                                static_cast<V>(v[3 * j + 1]), static_cast<V>(v[3 * j + 2]),
                                static_cast<S>(m[j]),
                                static_cast<int32_t>(j), 0};
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) pair<P>(xi, yi, zi, vxi, vyi, vzi, i, tile[k], eps2, A);
    }
    if (!has_q) return;
    if (!ok) {
#pragma unroll
        for (int k = 0; k < kOut; ++k) A.v[k] = __builtin_nan("");
    }
    if (gridDim.y == 1) {
        acc[3 * q] = A.v[0];
        acc[3 * q + 1] = A.v[1];
        acc[3 * q + 2] = A.v[2];
        jerk[3 * q] = A.v[3];
        jerk[3 * q + 1] = A.v[4];
        jerk[3 * q + 2] = A.v[5];
        pot[q] = A.v[6];
        return;
    }
    double* p = part + (static_cast<int64_t>(split) * n_active + q) * kOut;
#pragma unroll
    for (int k = 0; k < kOut; ++k) p[k] = A.v[k];
}

// The split partials of every active particle, added in split order.
__global__ __launch_bounds__(kWG) void noalloc_reduce_kernel(int32_t n_active, int32_t n_split,
                                                             const double* __restrict__ part, double* acc,
                                                             double* jerk, double* pot) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
    if (q >= n_active) return;
    double A[kOut];
    for (int k = 0; k < kOut; ++k) A[k] = part[q * kOut + k];
    for (int s = 1; s < n_split; ++s)
        for (int k = 0; k < kOut; ++k) A[k] += part[(static_cast<int64_t>(s) * n_active + q) * kOut + k];
    acc[3 * q] = A[0];
    acc[3 * q + 1] = A[1];
    acc[3 * q + 2] = A[2];
    jerk[3 * q] = A[3];
    jerk[3 * q + 1] = A[4];
    jerk[3 * q + 2] = A[5];
    pot[q] = A[6];
}

}  // namespace

extern "C" {

int ht_force_direct_noalloc(int32_t device, void* stream, int32_t precision, int32_t n, const double* d_x,
                            const double* d_v, const double* d_m, double eps2, int32_t n_active,
                            const int32_t* d_active, int32_t j_splits, double* d_acc, double* d_jerk,
                            double* d_pot) {
    if (precision != HT_PREC_FP64 && precision != HT_PREC_MIXED) return fail(HT_EINVAL, "unknown precision");
    if (device < 0 || device >= kMaxDevices) return fail(HT_EINVAL, "device %d outside [0, %d)", device, kMaxDevices);
    if (n < 1 || n_active < 0) return fail(HT_EINVAL, "n must be >= 1 and n_active >= 0");
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return fail(HT_EINVAL, "eps2 must be finite and >= 0");
    if (j_splits < 1 || j_splits > 65535) return fail(HT_EINVAL, "j_splits = %d outside [1, 65535]", j_splits);
    if (n_active == 0) return HT_OK;
    if (!d_x || !d_v || !d_m || !d_active || !d_acc || !d_jerk || !d_pot) return fail(HT_EINVAL, "NULL device array");
    const size_t need = j_splits > 1 ? static_cast<size_t>(j_splits) * static_cast<size_t>(n_active) * kOut * 8 : 0;
    if (need > kScratchBytes)
        return fail(HT_ERANGE, "%d splits of %d active particles need %zu bytes of scratch; the library holds %zu",
                    j_splits, n_active, need, kScratchBytes);
    double* part = nullptr;
    if (j_splits > 1) {
        int rc = scratch_on(device, &part);
        if (rc) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t per = (static_cast<int64_t>(n) + j_splits - 1) / j_splits;
    const dim3 grid(static_cast<unsigned>((n_active + kWG - 1) / kWG), static_cast<unsigned>(j_splits));
    if (precision == HT_PREC_FP64)
        noalloc_direct_kernel<PrecFp64><<<grid, kWG, 0, s>>>(n, d_x, d_v, d_m, eps2, n_active, d_active, per, part,
                                                             d_acc, d_jerk, d_pot);
    else
        noalloc_direct_kernel<PrecMixed><<<grid, kWG, 0, s>>>(n, d_x, d_v, d_m, eps2, n_active, d_active, per, part,
                                                              d_acc, d_jerk, d_pot);
    HT_HIP(hipGetLastError());
    if (j_splits > 1) {
        noalloc_reduce_kernel<<<(n_active + kWG - 1) / kWG, kWG, 0, s>>>(n_active, j_splits, part, d_acc, d_jerk,
                                                                         d_pot);
        HT_HIP(hipGetLastError());
    }
    return HT_OK;
}

}  // extern "C"
