// Step 1 of the tree/Hermite scheme on the device (Fukushige & Kawai,
// Section 2): Peano-Hilbert keys, the sorted particle order, the octree,
// node moments, groups and the interaction lists, computed from particles
// already resident in device memory.  The definitions are those of the host
// builder (include/htree_host.h), and the results are bit-identical to it:
// the same keys and order, the same node sums in the same order, the same
// opening test with the same roundings, the same lists in the same order.
//
// Layout of the work (one stream, synchronous entry point):
//   1. root cube from a min/max reduction; 63-bit keys; stable radix sort of
//      (key, index) pairs; the particle state gathered into key order.
//   2. the octree without a pointer walk.  With L_k the first level at which
//      particle k's key leaves particle k-1's cell, the cells that begin at
//      particle k are those of levels L_k ... E_k, and pre-order is the order
//      of (first particle, level).  Per-particle counts and three prefix sums
//      give every cell, node and group its pre-order number directly.
//   3. node moments, bottom-up: one launch per level from the deepest up, one
//      thread per node of that level adding its children's sums (or a leaf's
//      particles) in order, then the means.
//   4. lists: one work-group per group keeps the group's current cut through
//      the tree as an ordered array; every pass replaces each undecided cell
//      by its decision (the node, its particles, or its children), in place
//      and in order, so the final array is the pre-order list.
#include "htree_tree.h"
#include "wave_ops.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <string>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace {

constexpr int kAxisBits = 21;      // bits per axis of the key
constexpr int kDeepest = 21;       // deepest cell level
constexpr int kNoCellLevel = 22;   // L_k of a particle whose key equals its predecessor's
constexpr int kWG = 256;
constexpr int kListWG = 256;
constexpr int64_t kMaxN = int64_t(1) << 26;   // every cell count fits in int32 (<= 22 N)

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

#define HTD_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(HTD_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Cell {
    int32_t begin, end;   // particle range [begin, end) in key order
    int32_t skip;         // first cell after this cell's subtree (pre-order)
    int32_t node;         // node number, -1 for a single-particle cell
    int32_t level;
    int32_t split;        // 1 if the cell has children
    int32_t pad0, pad1;
};
static_assert(sizeof(Cell) == 32, "cell record");

struct Totals {           // written by the device after the prefix sums
    int32_t cells, nodes, groups, pad;
};

struct Counters {         // list phase
    unsigned long long staged;   // entries reserved in the staging array
    int32_t max_cut;             // largest cut that did not fit a work-group's scratch
    int32_t pad;
};

// ---------------------------------------------------------------- keys
__device__ inline uint64_t spread3(uint32_t v) {
    uint64_t s = v & 0x1fffffu;
    s = (s | s << 32) & 0x1f00000000ffffull;
    s = (s | s << 16) & 0x1f0000ff0000ffull;
    s = (s | s << 8) & 0x100f00f00f00f00full;
    s = (s | s << 4) & 0x10c30c30c30c30c3ull;
    s = (s | s << 2) & 0x1249249249249249ull;
    return s;
}

// Peano-Hilbert index of a lattice point (J. Skilling, "Programming the
// Hilbert curve", AIP Conf. Proc. 707, 2004): axes to transposed index, then
// the bits interleaved from the top with x first.
__device__ inline uint64_t ph_key(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t c0 = x, c1 = y, c2 = z;
    for (uint32_t q = 1u << (kAxisBits - 1); q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        {   // axis 0: invert or leave
            const uint32_t set = 0u - static_cast<uint32_t>((c0 & q) != 0);
            c0 ^= low & set;
        }
        {
            const uint32_t set = 0u - static_cast<uint32_t>((c1 & q) != 0);
            const uint32_t swap = (c0 ^ c1) & low & ~set;
            c0 ^= (low & set) | swap;
            c1 ^= swap;
        }
        {
            const uint32_t set = 0u - static_cast<uint32_t>((c2 & q) != 0);
            const uint32_t swap = (c0 ^ c2) & low & ~set;
            c0 ^= (low & set) | swap;
            c2 ^= swap;
        }
    }
    c1 ^= c0;
    c2 ^= c1;
    uint32_t flip = 0;
    for (uint32_t q = 1u << (kAxisBits - 1); q > 1; q >>= 1) flip ^= (q - 1) & (0u - static_cast<uint32_t>((c2 & q) != 0));
    c0 ^= flip;
    c1 ^= flip;
    c2 ^= flip;
    return (spread3(c0) << 2) | (spread3(c1) << 1) | spread3(c2);
}

__device__ inline double dmin(double a, double b) { return b < a ? b : a; }
__device__ inline double dmax(double a, double b) { return a < b ? b : a; }

// Per-block componentwise min and max of x (exact in any order).
__global__ __launch_bounds__(kWG) void bbox_partial_kernel(int64_t n, const double* __restrict__ x,
                                                           double* __restrict__ part) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = x[d];
    for (int64_t i = blockIdx.x * int64_t(kWG) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kWG)
        for (int d = 0; d < 3; ++d) {
            lo[d] = dmin(lo[d], x[3 * i + d]);
            hi[d] = dmax(hi[d], x[3 * i + d]);
        }
    __shared__ double s[6][kWG];
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = lo[d];
        s[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = dmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
                s[3 + d][threadIdx.x] = dmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

struct Root {
    double lo[3];
    double side;
    double scale;    // 2^21 / side
};

// Final reduction and the root cube: side is the smallest power of two above
// the largest extent (1 when all particles coincide).
__global__ __launch_bounds__(kWG) void bbox_final_kernel(int nb, const double* __restrict__ part, Root* root) {
    __shared__ double s[6][kWG];
    const int t = threadIdx.x;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = part[d];
        hi[d] = part[3 + d];
    }
    for (int b = t; b < nb; b += kWG)
        for (int d = 0; d < 3; ++d) {
            lo[d] = dmin(lo[d], part[6 * b + d]);
            hi[d] = dmax(hi[d], part[6 * b + 3 + d]);
        }
    for (int d = 0; d < 3; ++d) {
        s[d][t] = lo[d];
        s[3 + d][t] = hi[d];
    }
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int d = 0; d < 3; ++d) {
                s[d][t] = dmin(s[d][t], s[d][t + w]);
                s[3 + d][t] = dmax(s[3 + d][t], s[3 + d][t + w]);
            }
        __syncthreads();
    }
    if (t != 0) return;
    for (int d = 0; d < 3; ++d) {
        lo[d] = s[d][0];
        hi[d] = s[3 + d][0];
    }
    const double ext = dmax(dmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    double side = 1.0;
    if (ext > 0.0) {
        int e;
        frexp(ext, &e);
        side = ldexp(1.0, e);
    }
    for (int d = 0; d < 3; ++d) root->lo[d] = lo[d];
    root->side = side;
    root->scale = ldexp(1.0, kAxisBits) / side;
}

__global__ __launch_bounds__(kWG) void keys_kernel(int64_t n, const double* __restrict__ x, const Root* root,
                                                   uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
    const int64_t i = blockIdx.x * int64_t(kWG) + threadIdx.x;
    if (i >= n) return;
    const double qmax = ldexp(1.0, kAxisBits) - 1.0;
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double u = floor((x[3 * i + d] - root->lo[d]) * root->scale);
        u = dmin(dmax(u, 0.0), qmax);
        q[d] = static_cast<uint32_t>(u);
    }
    key[i] = ph_key(q[0], q[1], q[2]);
    idx[i] = static_cast<int32_t>(i);
}

// Particle state in key order, and L_k.
__global__ __launch_bounds__(kWG) void gather_kernel(int64_t n, const int32_t* __restrict__ perm32,
                                                     const uint64_t* __restrict__ key, const double* __restrict__ x,
                                                     const double* __restrict__ v, const double* __restrict__ a,
                                                     const double* __restrict__ j, const double* __restrict__ m,
                                                     int64_t* __restrict__ perm, double* __restrict__ sx,
                                                     double* __restrict__ sv, double* __restrict__ sa,
                                                     double* __restrict__ sj, double* __restrict__ sm,
                                                     int8_t* __restrict__ lev) {
    const int64_t k = blockIdx.x * int64_t(kWG) + threadIdx.x;
    if (k >= n) return;
    const int64_t o = perm32[k];
    perm[k] = o;
    sm[k] = m[o];
    for (int d = 0; d < 3; ++d) {
        sx[3 * k + d] = x[3 * o + d];
        sv[3 * k + d] = v[3 * o + d];
        sa[3 * k + d] = a[3 * o + d];
        sj[3 * k + d] = j[3 * o + d];
    }
    int L = 0;
    if (k > 0) {
        const uint64_t diff = key[k] ^ key[k - 1];
        // digit i (0-based from the top) holds bits 60-3i .. 62-3i; the keys part at level i+1
        L = diff == 0 ? kNoCellLevel : kDeepest - (63 - __clzll(diff)) / 3;
    }
    lev[k] = static_cast<int8_t>(L);
}

__device__ inline uint64_t level_mask(int level) {
    const int sh = 3 * (kDeepest - level);
    return sh >= 63 ? 0ull : (~0ull << sh);
}

// [b, e): the particles whose key shares key's first `level` digits.
__device__ inline void prefix_range(const uint64_t* __restrict__ key, int64_t n, uint64_t k, int level, int64_t* b,
                                    int64_t* e) {
    const uint64_t mask = level_mask(level);
    const uint64_t lo = k & mask, hi = lo | (~mask & 0x7fffffffffffffffull);
    int64_t l = 0, r = n;   // first key >= lo
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        if (key[mid] < lo) l = mid + 1; else r = mid;
    }
    *b = l;
    r = n;                  // first key > hi
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        if (key[mid] <= hi) l = mid + 1; else r = mid;
    }
    *e = l;
}

__device__ inline int64_t prefix_end(const uint64_t* __restrict__ key, int64_t n, int64_t from, uint64_t k,
                                     int level) {
    const uint64_t hi = (k & level_mask(level)) | (~level_mask(level) & 0x7fffffffffffffffull);
    int64_t l = from, r = n;
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        if (key[mid] <= hi) l = mid + 1; else r = mid;
    }
    return l;
}

// Whether cells begin at k, and their deepest level.
__device__ inline bool cells_at(const uint64_t* __restrict__ key, const int8_t* __restrict__ lev, int64_t n,
                                int n_leaf, int64_t k, int* Lk, int* Ek) {
    const int L = lev[k];
    if (L > kDeepest) return false;
    if (k > 0 && n_leaf > 1) {   // the parent cell must hold more than n_leaf particles
        int64_t b, e;
        prefix_range(key, n, key[k], L - 1, &b, &e);
        if (e - b <= n_leaf) return false;
    }
    int mk = kNoCellLevel;   // min L over the next n_leaf particles; 0 when they run out
    if (k + n_leaf >= n) {
        mk = 0;
    } else {
        for (int i = 1; i <= n_leaf; ++i) mk = min(mk, static_cast<int>(lev[k + i]));
    }
    *Lk = L;
    *Ek = max(L, min(kDeepest, mk));
    return true;
}

// Per particle: cells, nodes and the group that begin there.
__global__ __launch_bounds__(kWG) void count_kernel(int64_t n, int n_leaf, int n_crit,
                                                    const uint64_t* __restrict__ key, const int8_t* __restrict__ lev,
                                                    int32_t* __restrict__ n_cells, int32_t* __restrict__ n_nodes,
                                                    int32_t* __restrict__ gflag) {
    const int64_t k = blockIdx.x * int64_t(kWG) + threadIdx.x;
    if (k >= n) return;
    int L, E;
    int32_t nc = 0, nn = 0, g = 0;
    if (cells_at(key, lev, n, n_leaf, k, &L, &E)) {
        nc = E - L + 1;
        if (k + 1 < n) nn = max(0, min(E, static_cast<int>(lev[k + 1]) - 1) - L + 1);
        if (k == 0) {
            g = 1;
        } else {   // a group starts here unless the enclosing cell already qualifies
            int64_t b, e;
            prefix_range(key, n, key[k], L - 1, &b, &e);
            g = (e - b > n_crit) ? 1 : 0;
        }
    }
    n_cells[k] = nc;
    n_nodes[k] = nn;
    gflag[k] = g;
}

__global__ void totals_kernel(int64_t n, const int32_t* __restrict__ n_cells, const int32_t* __restrict__ cbase,
                              const int32_t* __restrict__ n_nodes, const int32_t* __restrict__ nbase,
                              const int32_t* __restrict__ gflag, const int32_t* __restrict__ gbase, Totals* t) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    t->cells = cbase[n - 1] + n_cells[n - 1];
    t->nodes = nbase[n - 1] + n_nodes[n - 1];
    t->groups = gbase[n - 1] + gflag[n - 1];
    t->pad = 0;
}

__global__ __launch_bounds__(kWG) void cells_kernel(int64_t n, int n_leaf, const uint64_t* __restrict__ key,
                                                    const int8_t* __restrict__ lev,
                                                    const int32_t* __restrict__ cbase,
                                                    const int32_t* __restrict__ nbase,
                                                    const int32_t* __restrict__ gflag,
                                                    const int32_t* __restrict__ gbase, const Totals* tot,
                                                    Cell* __restrict__ cell, int32_t* __restrict__ node_level,
                                                    int64_t* __restrict__ node_begin, int64_t* __restrict__ node_end,
                                                    int32_t* __restrict__ node_cell, int64_t* __restrict__ group_first) {
    const int64_t k = blockIdx.x * int64_t(kWG) + threadIdx.x;
    if (k == 0) group_first[tot->groups] = n;
    if (k >= n) return;
    int L, E;
    if (!cells_at(key, lev, n, n_leaf, k, &L, &E)) return;
    if (gflag[k]) group_first[gbase[k]] = k;
    const int32_t total = tot->cells;
    for (int l = L; l <= E; ++l) {
        const int64_t e = prefix_end(key, n, k, key[k], l);
        const int64_t cnt = e - k;
        Cell c;
        c.begin = static_cast<int32_t>(k);
        c.end = static_cast<int32_t>(e);
        c.skip = e < n ? cbase[e] : total;
        c.node = cnt >= 2 ? nbase[k] + (l - L) : -1;
        c.level = l;
        c.split = (cnt > n_leaf && l < kDeepest) ? 1 : 0;
        c.pad0 = c.pad1 = 0;
        cell[cbase[k] + (l - L)] = c;
        if (c.node >= 0) {
            node_level[c.node] = l;
            node_begin[c.node] = k;
            node_end[c.node] = e;
            node_cell[c.node] = cbase[k] + (l - L);
        }
    }
}

// Node moments, bottom-up, as the host builder defines them: a node's sums
// S = (m, m x[3], m v[3], m a[3], m jerk[3]) start from zero and add, for a
// split node, its children's S in key order (a single-particle child's S is
// 0 + its rounded products), otherwise its particles' rounded products in
// ascending order.  No fused multiply-add anywhere, so the bits match.  A
// child is one level deeper than its parent, so one launch per level, from
// the deepest up, sums every node of that level (at most eight children
// each, or the particles of a leaf).  raw holds S, 13 doubles per node.
#pragma clang fp contract(off)
__device__ inline void add_products(int64_t k, const double* __restrict__ sm, const double* __restrict__ sx,
                                    const double* __restrict__ sv, const double* __restrict__ sa,
                                    const double* __restrict__ sj, double (&u)[13]) {
    const double mk = sm[k];
    u[0] = u[0] + mk;
    for (int d = 0; d < 3; ++d) {
        u[1 + d] = u[1 + d] + mk * sx[3 * k + d];
        u[4 + d] = u[4 + d] + mk * sv[3 * k + d];
        u[7 + d] = u[7 + d] + mk * sa[3 * k + d];
        u[10 + d] = u[10 + d] + mk * sj[3 * k + d];
    }
}

__global__ __launch_bounds__(kWG) void node_sums_kernel(int32_t level, int32_t m_nodes,
                                                        const int32_t* __restrict__ node_level,
                                                        const int32_t* __restrict__ node_cell,
                                                        const Cell* __restrict__ cell, const double* __restrict__ sm,
                                                        const double* __restrict__ sx, const double* __restrict__ sv,
                                                        const double* __restrict__ sa, const double* __restrict__ sj,
                                                        double* __restrict__ raw) {
    const int32_t q = blockIdx.x * kWG + threadIdx.x;
    if (q >= m_nodes || node_level[q] != level) return;
    const int32_t ci = node_cell[q];
    const Cell c = cell[ci];
    double s[13];
    for (int r = 0; r < 13; ++r) s[r] = 0.0;
    if (c.split) {
        for (int32_t ch = ci + 1; ch < c.skip;) {
            const Cell cc = cell[ch];
            double u[13];
            if (cc.node >= 0) {
                for (int r = 0; r < 13; ++r) u[r] = raw[13 * int64_t(cc.node) + r];
            } else {
                for (int r = 0; r < 13; ++r) u[r] = 0.0;
                add_products(cc.begin, sm, sx, sv, sa, sj, u);
            }
            for (int r = 0; r < 13; ++r) s[r] = s[r] + u[r];
            ch = cc.skip;
        }
    } else {
        for (int64_t k = c.begin; k < c.end; ++k) add_products(k, sm, sx, sv, sa, sj, s);
    }
    for (int r = 0; r < 13; ++r) raw[13 * int64_t(q) + r] = s[r];
}

__global__ __launch_bounds__(kWG) void node_means_kernel(int32_t m_nodes, const double* __restrict__ raw,
                                                         double* __restrict__ om, double* __restrict__ ox,
                                                         double* __restrict__ ov, double* __restrict__ oa,
                                                         double* __restrict__ oj) {
    const int32_t q = blockIdx.x * kWG + threadIdx.x;
    if (q >= m_nodes) return;
    const double* u = raw + 13 * int64_t(q);
    const double M = u[0];
    om[q] = M;
    for (int d = 0; d < 3; ++d) {
        ox[3 * q + d] = u[1 + d] / M;
        ov[3 * q + d] = u[4 + d] / M;
        oa[3 * q + d] = u[7 + d] / M;
        oj[3 * q + d] = u[10 + d] / M;
    }
}
#pragma clang fp contract(on)

// ---------------------------------------------------------------- lists
struct ListArgs {
    int64_t n;
    int32_t n_groups;
    int32_t cut_cap;
    const Cell* cell;
    const double* node_x;
    const double* sx;
    const int64_t* group_first;
    int32_t* cut;             // per work-group: 4 arrays of cut_cap int32
    int32_t* stage;
    int64_t stage_cap;
    int32_t* glen;
    int64_t* gstage;
    Counters* ctr;
    double theta2;
    double s2[kDeepest + 1];
};

enum : int32_t { kKeep = 0, kParticle = 1, kNode = 2, kParticles = 3, kChildren = 4 };

// Exclusive prefix sum over the work-group; returns the total.
__device__ inline int32_t wg_scan(int32_t v, int32_t* excl, int32_t* s_wave) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t x = wave_ops::scan_inclusive(v);
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < kListWG / 64; ++w) {
        const int32_t s = s_wave[w];
        if (w < wave) before += s;
        total += s;
    }
    *excl = before + x - v;
    __syncthreads();
    return total;
}

#pragma clang fp contract(off)
// The opening test of the host builder: accept a node iff side^2 < theta^2 d^2,
// d the distance from its centre of mass to the group's box.
__device__ inline int32_t decide(const ListArgs& A, int32_t c, int64_t gb, int64_t ge, const double* lo,
                                 const double* hi, int32_t* cnt) {
    const Cell cl = A.cell[c];
    const bool overlaps = cl.begin < ge && gb < cl.end;
    if (!overlaps) {
        if (cl.end - cl.begin == 1) {
            *cnt = 1;
            return kParticle;
        }
        const double* X = A.node_x + 3 * int64_t(cl.node);
        double gap[3];
        for (int d = 0; d < 3; ++d) {
            const double u = dmax(lo[d] - X[d], X[d] - hi[d]);
            gap[d] = dmax(u, 0.0);
        }
        const double d2 = (gap[0] * gap[0] + gap[1] * gap[1]) + gap[2] * gap[2];
        if (A.s2[cl.level] < A.theta2 * d2) {
            *cnt = 1;
            return kNode;
        }
    }
    if (cl.split) {
        int32_t k = 0;
        for (int32_t ch = c + 1; ch < cl.skip; ch = A.cell[ch].skip) ++k;
        *cnt = k;
        return kChildren;
    }
    *cnt = cl.end - cl.begin;
    return kParticles;
}
#pragma clang fp contract(on)

__global__ __launch_bounds__(kListWG) void lists_kernel(ListArgs A) {
    __shared__ int32_t s_wave[kListWG / 64];
    __shared__ double s_box[6][kListWG];
    __shared__ int32_t s_flag[2];
    __shared__ unsigned long long s_off;
    const int t = threadIdx.x;
    int32_t* bufA = A.cut + int64_t(blockIdx.x) * 4 * A.cut_cap;
    int32_t* bufB = bufA + A.cut_cap;
    int32_t* pos = bufB + A.cut_cap;
    int32_t* dec = pos + A.cut_cap;
    for (int32_t g = blockIdx.x; g < A.n_groups; g += gridDim.x) {
        const int64_t gb = A.group_first[g], ge = A.group_first[g + 1];
        // group box: componentwise min and max of the members' positions
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = A.sx[3 * gb + d];
        for (int64_t k = gb + t; k < ge; k += kListWG)
            for (int d = 0; d < 3; ++d) {
                lo[d] = dmin(lo[d], A.sx[3 * k + d]);
                hi[d] = dmax(hi[d], A.sx[3 * k + d]);
            }
        for (int d = 0; d < 3; ++d) {
            s_box[d][t] = lo[d];
            s_box[3 + d][t] = hi[d];
        }
        __syncthreads();
        for (int w = kListWG / 2; w > 0; w >>= 1) {
            if (t < w)
                for (int d = 0; d < 3; ++d) {
                    s_box[d][t] = dmin(s_box[d][t], s_box[d][t + w]);
                    s_box[3 + d][t] = dmax(s_box[3 + d][t], s_box[3 + d][t + w]);
                }
            __syncthreads();
        }
        for (int d = 0; d < 3; ++d) {
            lo[d] = s_box[d][0];
            hi[d] = s_box[3 + d][0];
        }
        __syncthreads();

        int32_t* cur = bufA;
        int32_t* nxt = bufB;
        if (t == 0) {
            cur[0] = -1;   // the root cell, undecided
            s_flag[0] = s_flag[1] = 0;
        }
        int32_t len = 1;
        bool overflow = false;
        __syncthreads();
        for (int it = 0;; ++it) {
            // pass 1: decisions and output counts, chunk by chunk with a running offset
            int32_t carry = 0;
            bool more = false;
            for (int32_t s = 0; s < len; s += kListWG) {
                const int32_t i = s + t;
                int32_t cnt = 0;
                if (i < len) {
                    const int32_t v = cur[i];
                    int32_t d = kKeep;
                    if (v >= 0) {
                        cnt = 1;
                    } else {
                        d = decide(A, -v - 1, gb, ge, lo, hi, &cnt);
                        if (d == kChildren) more = true;
                    }
                    dec[i] = d;
                }
                int32_t excl;
                const int32_t tot = wg_scan(cnt, &excl, s_wave);
                if (i < len) pos[i] = carry + excl;
                carry += tot;
            }
            if (more) s_flag[it & 1] = 1;
            const int32_t new_len = carry;
            if (new_len > A.cut_cap) {
                if (t == 0) atomicMax(&A.ctr->max_cut, new_len);
                overflow = true;
                break;
            }
            __syncthreads();
            // every thread has read the other flag slot (end of the previous pass) before this barrier
            if (t == 0) s_flag[(it + 1) & 1] = 0;
            // pass 2: write every element's output at its offset, in order
            for (int32_t i = t; i < len; i += kListWG) {
                const int32_t v = cur[i];
                int32_t p = pos[i];
                switch (dec[i]) {
                    case kKeep: nxt[p] = v; break;
                    case kParticle: nxt[p] = A.cell[-v - 1].begin; break;
                    case kNode: nxt[p] = static_cast<int32_t>(A.n) + A.cell[-v - 1].node; break;
                    case kParticles: {
                        const Cell cl = A.cell[-v - 1];
                        for (int32_t k = cl.begin; k < cl.end; ++k) nxt[p++] = k;
                        break;
                    }
                    default: {
                        const int32_t c = -v - 1;
                        const int32_t stop = A.cell[c].skip;
                        for (int32_t ch = c + 1; ch < stop; ch = A.cell[ch].skip) nxt[p++] = -ch - 1;
                        break;
                    }
                }
            }
            __syncthreads();
            const bool again = s_flag[it & 1] != 0;
            int32_t* tmp = cur;
            cur = nxt;
            nxt = tmp;
            len = new_len;
            if (!again) break;
        }
        // stage the finished list
        if (t == 0) s_off = overflow ? ~0ull : atomicAdd(&A.ctr->staged, static_cast<unsigned long long>(len));
        __syncthreads();
        const unsigned long long off = s_off;
        const bool fits = !overflow && off + static_cast<unsigned long long>(len) <= static_cast<unsigned long long>(A.stage_cap);
        if (fits)
            for (int32_t i = t; i < len; i += kListWG) A.stage[off + i] = cur[i];
        if (t == 0) {
            A.glen[g] = overflow ? 0 : len;
            A.gstage[g] = fits ? static_cast<int64_t>(off) : -1;
        }
        __syncthreads();
    }
}

// CSR copy: group g's staged list to entries[list_off[g] ...].
__global__ __launch_bounds__(kWG) void csr_kernel(int32_t n_groups, const int64_t* __restrict__ list_off,
                                                  const int64_t* __restrict__ gstage,
                                                  const int32_t* __restrict__ stage, int32_t* __restrict__ entries) {
    for (int32_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int64_t b = list_off[g], len = list_off[g + 1] - b, s = gstage[g];
        for (int64_t i = threadIdx.x; i < len; i += kWG) entries[b + i] = stage[s + i];
    }
}

__global__ void glen_to_off_kernel(int32_t n_groups, const int32_t* __restrict__ glen, int64_t* __restrict__ len64) {
    const int32_t g = blockIdx.x * kWG + threadIdx.x;
    if (g < n_groups) len64[g] = glen[g];
    if (g == n_groups) len64[g] = 0;
}

template <class T>
struct DevBuf {
    T* p = nullptr;
    int64_t cap = 0;
    int grow(int64_t need) {
        if (need <= cap) return 0;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const int64_t want = need + need / 4 + 16;
        if (hipMalloc(&p, sizeof(T) * static_cast<size_t>(want)) != hipSuccess) {
            p = nullptr;
            return fail(HTD_ENOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * want));
        }
        cap = want;
        return 0;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

inline unsigned blocks_for(int64_t n, int wg) { return static_cast<unsigned>((n + wg - 1) / wg); }

}  // namespace

struct htd_tree {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_max = 0;
    // per particle
    DevBuf<uint64_t> key_in, key;
    DevBuf<int32_t> idx_in, idx;
    DevBuf<int64_t> perm;
    DevBuf<double> sx, sv, sa, sj, sm;
    DevBuf<int8_t> lev;
    DevBuf<int32_t> ncell, cbase, nnode, nbase, gflag, gbase;
    DevBuf<char> tmp;
    DevBuf<double> part;
    DevBuf<Root> root;
    DevBuf<Totals> tot;
    // cells and nodes
    DevBuf<Cell> cell;
    DevBuf<double> nm, nx, nv, na, nj;
    DevBuf<int32_t> nlev, ncid;   // per node: level, cell index
    DevBuf<double> nraw;            // per node: the 13 sums of its moments
    DevBuf<int64_t> nbeg, nend;
    // groups and lists
    DevBuf<int64_t> group_first, list_off, gstage, glen64;
    DevBuf<int32_t> glen, cut, stage, entries;
    DevBuf<Counters> ctr;
    int32_t cut_cap = 1 << 15;
    int n_list_wg = 1024;
    // results of the last build
    int64_t n = 0, C = 0, M = 0, G = 0, L = 0;
    Root root_h{};
    hipEvent_t ev[8] = {};
    float phase_ms[7] = {};
    bool built = false;
};

namespace {

// Temporary storage of the library primitives, sized once per build before
// anything is queued (freeing a buffer a queued primitive still uses would
// be unsafe).  Node counts are bounded by 22 n (a chain of single-child
// cells down to the deepest level per particle).
int reserve_tmp(htd_tree* t, int64_t n) {
    size_t a = 0, b = 0, c = 0;
    HTD_HIP(rocprim::radix_sort_pairs(nullptr, a, t->key_in.p, t->key.p, t->idx_in.p, t->idx.p,
                                      static_cast<size_t>(n), 0, 63, t->stream));
    HTD_HIP(rocprim::exclusive_scan(nullptr, b, t->ncell.p, t->cbase.p, int32_t(0), static_cast<size_t>(22 * n),
                                    rocprim::plus<int32_t>(), t->stream));
    HTD_HIP(rocprim::exclusive_scan(nullptr, c, t->glen64.p, t->list_off.p, int64_t(0), static_cast<size_t>(n + 1),
                                    rocprim::plus<int64_t>(), t->stream));
    return t->tmp.grow(static_cast<int64_t>(std::max(a, std::max(b, c))));
}

int scan_i32(htd_tree* t, const int32_t* in, int32_t* out, int64_t n) {
    size_t bytes = static_cast<size_t>(t->tmp.cap);
    HTD_HIP(rocprim::exclusive_scan(t->tmp.p, bytes, in, out, int32_t(0), static_cast<size_t>(n),
                                    rocprim::plus<int32_t>(), t->stream));
    return 0;
}

int scan_i64(htd_tree* t, const int64_t* in, int64_t* out, int64_t n) {
    size_t bytes = static_cast<size_t>(t->tmp.cap);
    HTD_HIP(rocprim::exclusive_scan(t->tmp.p, bytes, in, out, int64_t(0), static_cast<size_t>(n),
                                    rocprim::plus<int64_t>(), t->stream));
    return 0;
}

int grow_particles(htd_tree* t, int64_t n) {
    int rc = 0;
    if ((rc = t->key_in.grow(n)) || (rc = t->key.grow(n)) || (rc = t->idx_in.grow(n)) || (rc = t->idx.grow(n)) ||
        (rc = t->perm.grow(n)) || (rc = t->sx.grow(3 * n)) || (rc = t->sv.grow(3 * n)) || (rc = t->sa.grow(3 * n)) ||
        (rc = t->sj.grow(3 * n)) || (rc = t->sm.grow(n)) || (rc = t->lev.grow(n)) || (rc = t->ncell.grow(n)) ||
        (rc = t->cbase.grow(n)) || (rc = t->nnode.grow(n)) || (rc = t->nbase.grow(n)) || (rc = t->gflag.grow(n)) ||
        (rc = t->gbase.grow(n)) || (rc = t->part.grow(6 * 1024)) || (rc = t->root.grow(1)) || (rc = t->tot.grow(1)) ||
        (rc = t->ctr.grow(1)) || (rc = t->group_first.grow(n + 1)) ||
        (rc = t->list_off.grow(n + 1)) ||
        (rc = t->gstage.grow(n + 1)) || (rc = t->glen64.grow(n + 1)) || (rc = t->glen.grow(n + 1)))
        return rc;
    return 0;
}

int run_lists(htd_tree* t, const ListArgs& base, int32_t* max_cut, unsigned long long* staged) {
    ListArgs A = base;
    A.cut = t->cut.p;
    A.cut_cap = t->cut_cap;
    A.stage = t->stage.p;
    A.stage_cap = t->stage.cap;
    A.ctr = t->ctr.p;
    HTD_HIP(hipMemsetAsync(t->ctr.p, 0, sizeof(Counters), t->stream));
    const int wg = static_cast<int>(std::min<int64_t>(t->G, t->n_list_wg));
    lists_kernel<<<wg, kListWG, 0, t->stream>>>(A);
    HTD_HIP(hipGetLastError());
    Counters c{};
    HTD_HIP(hipMemcpyAsync(&c, t->ctr.p, sizeof c, hipMemcpyDeviceToHost, t->stream));
    HTD_HIP(hipStreamSynchronize(t->stream));
    *max_cut = c.max_cut;
    *staged = c.staged;
    return 0;
}

int build(htd_tree* t, int64_t n, const double* x, const double* v, const double* a, const double* jerk,
          const double* m, int n_leaf, int n_crit, double theta) {
    hipStream_t s = t->stream;
    if (int rc = grow_particles(t, n)) return rc;
    if (int rc = reserve_tmp(t, n)) return rc;
    HTD_HIP(hipEventRecord(t->ev[0], s));
    // 1. root cube, keys, sort, gather
    const int nb = static_cast<int>(std::min<int64_t>(1024, std::max<int64_t>(1, blocks_for(n, kWG))));
    bbox_partial_kernel<<<nb, kWG, 0, s>>>(n, x, t->part.p);
    bbox_final_kernel<<<1, kWG, 0, s>>>(nb, t->part.p, t->root.p);
    keys_kernel<<<blocks_for(n, kWG), kWG, 0, s>>>(n, x, t->root.p, t->key_in.p, t->idx_in.p);
    HTD_HIP(hipGetLastError());
    HTD_HIP(hipEventRecord(t->ev[1], s));
    {
        size_t bytes = static_cast<size_t>(t->tmp.cap);
        HTD_HIP(rocprim::radix_sort_pairs(t->tmp.p, bytes, t->key_in.p, t->key.p, t->idx_in.p, t->idx.p,
                                          static_cast<size_t>(n), 0, 63, s));
    }
    HTD_HIP(hipEventRecord(t->ev[2], s));
    gather_kernel<<<blocks_for(n, kWG), kWG, 0, s>>>(n, t->idx.p, t->key.p, x, v, a, jerk, m, t->perm.p, t->sx.p,
                                                     t->sv.p, t->sa.p, t->sj.p, t->sm.p, t->lev.p);
    // 2. cells, nodes and groups
    count_kernel<<<blocks_for(n, kWG), kWG, 0, s>>>(n, n_leaf, n_crit, t->key.p, t->lev.p, t->ncell.p, t->nnode.p,
                                                    t->gflag.p);
    HTD_HIP(hipGetLastError());
    if (int rc = scan_i32(t, t->ncell.p, t->cbase.p, n)) return rc;
    if (int rc = scan_i32(t, t->nnode.p, t->nbase.p, n)) return rc;
    if (int rc = scan_i32(t, t->gflag.p, t->gbase.p, n)) return rc;
    totals_kernel<<<1, 64, 0, s>>>(n, t->ncell.p, t->cbase.p, t->nnode.p, t->nbase.p, t->gflag.p, t->gbase.p,
                                   t->tot.p);
    Totals tot{};
    HTD_HIP(hipMemcpyAsync(&tot, t->tot.p, sizeof tot, hipMemcpyDeviceToHost, s));
    HTD_HIP(hipMemcpyAsync(&t->root_h, t->root.p, sizeof(Root), hipMemcpyDeviceToHost, s));
    HTD_HIP(hipStreamSynchronize(s));
    t->C = tot.cells;
    t->M = tot.nodes;
    t->G = tot.groups;
    if (t->C < 1 || t->G < 1) return fail(HTD_EHIP, "tree construction produced no cells");
    int rc = 0;
    const int64_t M1 = std::max<int64_t>(t->M, 1);
    if ((rc = t->cell.grow(t->C)) || (rc = t->nm.grow(M1)) || (rc = t->nx.grow(3 * M1)) ||
        (rc = t->nv.grow(3 * M1)) || (rc = t->na.grow(3 * M1)) || (rc = t->nj.grow(3 * M1)) ||
        (rc = t->nlev.grow(M1)) || (rc = t->ncid.grow(M1)) || (rc = t->nraw.grow(13 * M1)) ||
        (rc = t->nbeg.grow(M1)) || (rc = t->nend.grow(M1)))
        return rc;
    cells_kernel<<<blocks_for(n, kWG), kWG, 0, s>>>(n, n_leaf, t->key.p, t->lev.p, t->cbase.p, t->nbase.p,
                                                    t->gflag.p, t->gbase.p, t->tot.p, t->cell.p, t->nlev.p,
                                                    t->nbeg.p, t->nend.p, t->ncid.p, t->group_first.p);
    HTD_HIP(hipGetLastError());
    HTD_HIP(hipEventRecord(t->ev[3], s));
    // 3. node moments
    if (t->M > 0) {
        const int32_t Mi = static_cast<int32_t>(t->M);
        for (int level = kDeepest; level >= 0; --level)
            node_sums_kernel<<<blocks_for(Mi, kWG), kWG, 0, s>>>(level, Mi, t->nlev.p, t->ncid.p, t->cell.p, t->sm.p,
                                                                 t->sx.p, t->sv.p, t->sa.p, t->sj.p, t->nraw.p);
        node_means_kernel<<<blocks_for(Mi, kWG), kWG, 0, s>>>(Mi, t->nraw.p, t->nm.p, t->nx.p, t->nv.p, t->na.p,
                                                              t->nj.p);
        HTD_HIP(hipGetLastError());
    }
    HTD_HIP(hipEventRecord(t->ev[4], s));
    // 4. lists
    ListArgs A{};
    A.n = n;
    A.n_groups = static_cast<int32_t>(t->G);
    A.cell = t->cell.p;
    A.node_x = t->nx.p;
    A.sx = t->sx.p;
    A.group_first = t->group_first.p;
    A.glen = t->glen.p;
    A.gstage = t->gstage.p;
    A.theta2 = theta * theta;
    for (int l = 0; l <= kDeepest; ++l) {
        const double sl = std::ldexp(t->root_h.side, -l);
        A.s2[l] = sl * sl;
    }
    const int wg = static_cast<int>(std::min<int64_t>(t->G, t->n_list_wg));
    if ((rc = t->cut.grow(int64_t(wg) * 4 * t->cut_cap))) return rc;
    if ((rc = t->stage.grow(std::max<int64_t>(t->stage.cap, 64 * n)))) return rc;
    for (int attempt = 0;; ++attempt) {
        int32_t max_cut = 0;
        unsigned long long staged = 0;
        if ((rc = run_lists(t, A, &max_cut, &staged))) return rc;
        if (max_cut == 0 && staged <= static_cast<unsigned long long>(t->stage.cap)) {
            t->L = static_cast<int64_t>(staged);
            break;
        }
        if (attempt >= 3) return fail(HTD_ERANGE, "interaction lists did not fit after %d attempts", attempt + 1);
        if (max_cut > 0) {   // a group's cut outgrew the per-work-group scratch
            if (int64_t(max_cut) > INT32_MAX / 2) return fail(HTD_ERANGE, "a group's list exceeds 2^30 entries");
            t->cut_cap = std::max<int32_t>(t->cut_cap, max_cut + max_cut / 4);
            t->cut.release();
            if ((rc = t->cut.grow(int64_t(wg) * 4 * t->cut_cap))) return rc;
        }
        if (staged > static_cast<unsigned long long>(t->stage.cap)) {
            t->stage.release();
            if ((rc = t->stage.grow(static_cast<int64_t>(staged)))) return rc;
        }
    }
    HTD_HIP(hipEventRecord(t->ev[5], s));
    const int32_t Gi = static_cast<int32_t>(t->G);
    glen_to_off_kernel<<<blocks_for(int64_t(Gi) + 1, kWG), kWG, 0, s>>>(Gi, t->glen.p, t->glen64.p);
    if ((rc = scan_i64(t, t->glen64.p, t->list_off.p, int64_t(Gi) + 1))) return rc;
    if ((rc = t->entries.grow(std::max<int64_t>(t->L, 1)))) return rc;
    csr_kernel<<<std::min(Gi, 4096), kWG, 0, s>>>(Gi, t->list_off.p, t->gstage.p, t->stage.p, t->entries.p);
    HTD_HIP(hipGetLastError());
    HTD_HIP(hipEventRecord(t->ev[6], s));
    HTD_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < 6; ++i) HTD_HIP(hipEventElapsedTime(&t->phase_ms[i], t->ev[i], t->ev[i + 1]));
    HTD_HIP(hipEventElapsedTime(&t->phase_ms[6], t->ev[0], t->ev[6]));
    t->n = n;
    t->built = true;
    return 0;
}

template <class T>
int copy_out(T* dst, const T* src, int64_t count, hipStream_t s) {
    if (!dst || count <= 0) return 0;
    HTD_HIP(hipMemcpyAsync(dst, src, sizeof(T) * static_cast<size_t>(count), hipMemcpyDeviceToHost, s));
    return 0;
}

}  // namespace

extern "C" {

const char* htd_last_error(void) { return g_err.c_str(); }

int htd_create(htd_tree** out, int32_t device, void* stream, int64_t n_max) {
    if (!out) return fail(HTD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_max < 1 || n_max > kMaxN) return fail(HTD_EINVAL, "n_max %lld outside [1, 2^26]", (long long)n_max);
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(HTD_EHIP, "no HIP device");
    if (device < 0 || device >= count) return fail(HTD_EINVAL, "device %d outside [0, %d)", device, count);
    HTD_HIP(hipSetDevice(device));
    htd_tree* t = new (std::nothrow) htd_tree();
    if (!t) return fail(HTD_ENOMEM, "host allocation failed");
    t->device = device;
    t->stream = static_cast<hipStream_t>(stream);
    t->n_max = n_max;
    for (auto& e : t->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            htd_destroy(t);
            return fail(HTD_EHIP, "hipEventCreate failed");
        }
    if (int rc = grow_particles(t, n_max)) {
        htd_destroy(t);
        return rc;
    }
    *out = t;
    return 0;
}

int htd_destroy(htd_tree* t) {
    if (!t) return 0;
    (void)hipSetDevice(t->device);
    if (t->stream) (void)hipStreamSynchronize(t->stream);
    else (void)hipDeviceSynchronize();
    for (auto& e : t->ev)
        if (e) (void)hipEventDestroy(e);
    t->key_in.release(); t->key.release(); t->idx_in.release(); t->idx.release(); t->perm.release();
    t->sx.release(); t->sv.release(); t->sa.release(); t->sj.release(); t->sm.release(); t->lev.release();
    t->ncell.release(); t->cbase.release(); t->nnode.release(); t->nbase.release(); t->gflag.release();
    t->gbase.release(); t->tmp.release(); t->part.release(); t->root.release(); t->tot.release();
    t->cell.release(); t->nm.release(); t->nx.release(); t->nv.release(); t->na.release(); t->nj.release();
    t->nlev.release(); t->ncid.release(); t->nraw.release(); t->nbeg.release();
    t->nend.release(); t->group_first.release(); t->list_off.release(); t->gstage.release(); t->glen64.release();
    t->glen.release(); t->cut.release(); t->stage.release(); t->entries.release(); t->ctr.release();
    delete t;
    return 0;
}

int htd_build(htd_tree* t, int64_t n, const double* d_x, const double* d_v, const double* d_a, const double* d_jerk,
              const double* d_m, int32_t n_leaf, int32_t n_crit, double theta) {
    if (!t) return fail(HTD_EINVAL, "tree is NULL");
    if (n < 1 || n > t->n_max) return fail(HTD_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)t->n_max);
    if (!d_x || !d_v || !d_a || !d_jerk || !d_m) return fail(HTD_EINVAL, "a particle array is NULL");
    if (n_leaf < 1 || n_crit < 1) return fail(HTD_EINVAL, "n_leaf and n_crit must be positive");
    if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(HTD_EINVAL, "theta must be finite and >= 0");
    HTD_HIP(hipSetDevice(t->device));
    t->built = false;
    return build(t, n, d_x, d_v, d_a, d_jerk, d_m, n_leaf, n_crit, theta);
}

int htd_sizes(const htd_tree* t, int64_t* n_node, int64_t* n_group, int64_t* n_entries, int64_t* n_cell) {
    if (!t) return fail(HTD_EINVAL, "tree is NULL");
    if (!t->built) return fail(HTD_ESTATE, "no successful build");
    if (n_node) *n_node = t->M;
    if (n_group) *n_group = t->G;
    if (n_entries) *n_entries = t->L;
    if (n_cell) *n_cell = t->C;
    return 0;
}

int htd_root(const htd_tree* t, double* lo, double* side) {
    if (!t) return fail(HTD_EINVAL, "tree is NULL");
    if (!t->built) return fail(HTD_ESTATE, "no successful build");
    if (lo)
        for (int d = 0; d < 3; ++d) lo[d] = t->root_h.lo[d];
    if (side) *side = t->root_h.side;
    return 0;
}

int htd_get(const htd_tree* t, int64_t* perm, uint64_t* keys, double* node_m, double* node_x, double* node_v,
            double* node_a, double* node_j, int32_t* node_level, int64_t* node_begin, int64_t* node_end,
            int64_t* group_first, int64_t* list_off, int32_t* entries) {
    if (!t) return fail(HTD_EINVAL, "tree is NULL");
    if (!t->built) return fail(HTD_ESTATE, "no successful build");
    HTD_HIP(hipSetDevice(t->device));
    hipStream_t s = t->stream;
    int rc = 0;
    if ((rc = copy_out(perm, t->perm.p, t->n, s)) || (rc = copy_out(keys, t->key.p, t->n, s)) ||
        (rc = copy_out(node_m, t->nm.p, t->M, s)) || (rc = copy_out(node_x, t->nx.p, 3 * t->M, s)) ||
        (rc = copy_out(node_v, t->nv.p, 3 * t->M, s)) || (rc = copy_out(node_a, t->na.p, 3 * t->M, s)) ||
        (rc = copy_out(node_j, t->nj.p, 3 * t->M, s)) || (rc = copy_out(node_level, t->nlev.p, t->M, s)) ||
        (rc = copy_out(node_begin, t->nbeg.p, t->M, s)) || (rc = copy_out(node_end, t->nend.p, t->M, s)) ||
        (rc = copy_out(group_first, t->group_first.p, t->G + 1, s)) ||
        (rc = copy_out(list_off, t->list_off.p, t->G + 1, s)) || (rc = copy_out(entries, t->entries.p, t->L, s)))
        return rc;
    HTD_HIP(hipStreamSynchronize(s));
    return 0;
}

int htd_device_view(const htd_tree* t, htd_view* out) {
    if (!t || !out) return fail(HTD_EINVAL, "NULL argument");
    if (!t->built) return fail(HTD_ESTATE, "no successful build");
    out->perm = t->perm.p;
    out->keys = t->key.p;
    out->x = t->sx.p;
    out->v = t->sv.p;
    out->a = t->sa.p;
    out->jerk = t->sj.p;
    out->m = t->sm.p;
    out->node_m = t->nm.p;
    out->node_x = t->nx.p;
    out->node_v = t->nv.p;
    out->node_a = t->na.p;
    out->node_j = t->nj.p;
    out->group_first = t->group_first.p;
    out->list_off = t->list_off.p;
    out->entries = t->entries.p;
    return 0;
}

int htd_phase_ms(const htd_tree* t, double* ms) {
    if (!t || !ms) return fail(HTD_EINVAL, "NULL argument");
    if (!t->built) return fail(HTD_ESTATE, "no successful build");
    for (int i = 0; i < 7; ++i) ms[i] = t->phase_ms[i];
    return 0;
}

int htd_device_bytes(const htd_tree* t, size_t* bytes) {
    if (!t || !bytes) return fail(HTD_EINVAL, "NULL argument");
    size_t b = 0;
    auto add = [&](const auto& buf) { b += sizeof(*buf.p) * static_cast<size_t>(buf.cap); };
    add(t->key_in), add(t->key), add(t->idx_in), add(t->idx), add(t->perm);
    add(t->sx), add(t->sv), add(t->sa), add(t->sj), add(t->sm), add(t->lev);
    add(t->ncell), add(t->cbase), add(t->nnode), add(t->nbase), add(t->gflag), add(t->gbase);
    add(t->tmp), add(t->part), add(t->root), add(t->tot), add(t->cell);
    add(t->nm), add(t->nx), add(t->nv), add(t->na), add(t->nj), add(t->nlev), add(t->ncid), add(t->nraw);
    add(t->nbeg), add(t->nend), add(t->group_first), add(t->list_off), add(t->gstage), add(t->glen64);
    add(t->glen), add(t->cut), add(t->stage), add(t->entries), add(t->ctr);
    *bytes = b;
    return 0;
}

}  // extern "C"
