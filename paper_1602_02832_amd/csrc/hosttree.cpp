// Host side of the tree/Hermite scheme (Fukushige & Kawai, Section 2):
// step 1 (tree, groups, interaction lists at every tree time) and the host's
// share of steps 2, 6 and 7 (active-set selection, Hermite corrector, block
// timesteps).  See include/htree_host.h for the exact definitions.
//
// Must be compiled with -ffp-contract=off: node moments and the opening test
// are specified operation by operation so that the lists are reproducible.
#include "htree_host.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <vector>

namespace {

constexpr int kAxisBits = 21;  // bits per axis of the Peano-Hilbert key
constexpr int kDeepest = 21;   // deepest cell level

// Spread the low 21 bits of v so that bit k lands on bit 3k.
inline uint64_t spread3(uint32_t v) {
    uint64_t s = v & 0x1fffffu;
    s = (s | s << 32) & 0x1f00000000ffffull;
    s = (s | s << 16) & 0x1f0000ff0000ffull;
    s = (s | s << 8) & 0x100f00f00f00f00full;
    s = (s | s << 4) & 0x10c30c30c30c30c3ull;
    s = (s | s << 2) & 0x1249249249249249ull;
    return s;
}

// Peano-Hilbert index of a lattice point, following J. Skilling,
// "Programming the Hilbert curve" (AIP Conf. Proc. 707, 2004): convert the
// coordinates to the transposed index (inverse-undo then Gray code), here
// written without branches, then interleave x, y, z bits from the top.
inline uint64_t ph_key(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t c[3] = {x, y, z};
    for (uint32_t q = 1u << (kAxisBits - 1); q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (int d = 0; d < 3; ++d) {
            const uint32_t set = 0u - static_cast<uint32_t>((c[d] & q) != 0);
            const uint32_t swap = (c[0] ^ c[d]) & low & ~set;
            c[0] ^= (low & set) | swap;
            c[d] ^= swap;
        }
    }
    c[1] ^= c[0];
    c[2] ^= c[1];
    uint32_t flip = 0;
    for (uint32_t q = 1u << (kAxisBits - 1); q > 1; q >>= 1)
        flip ^= (q - 1) & (0u - static_cast<uint32_t>((c[2] & q) != 0));
    c[0] ^= flip;
    c[1] ^= flip;
    c[2] ^= flip;
    return (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
}

// Stable LSD radix sort of 64-bit keys carrying their original index; since
// the input is in index order this sorts by (key, index).
void radix_sort(std::vector<uint64_t>& key, std::vector<int64_t>& idx) {
    const size_t n = key.size();
    std::vector<uint64_t> k2(n);
    std::vector<int64_t> i2(n);
    for (int pass = 0; pass < 8; ++pass) {
        const int sh = 8 * pass;
        size_t cnt[257] = {0};
        for (size_t i = 0; i < n; ++i) cnt[((key[i] >> sh) & 255u) + 1]++;
        if (cnt[((key[0] >> sh) & 255u) + 1] == n) continue;  // digit constant: pass is identity
        for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
        for (size_t i = 0; i < n; ++i) {
            const size_t p = cnt[(key[i] >> sh) & 255u]++;
            k2[p] = key[i];
            i2[p] = idx[i];
        }
        key.swap(k2);
        idx.swap(i2);
    }
}

struct Cell {
    int32_t level;
    int32_t split;
    int64_t begin, end;
    int64_t skip;    // index of the first cell after this cell's subtree (pre-order)
    int64_t parent;
    int64_t node;    // node number, -1 when the cell holds a single particle
};

}  // namespace

struct htb_tree {
    int64_t n = 0;
    std::vector<int64_t> perm;
    std::vector<uint64_t> key;
    std::vector<Cell> cell;
    std::vector<int64_t> node_cell;
    std::vector<double> nm, nx, nv, na, nj;
    std::vector<int64_t> group_first, list_off;
    std::vector<int32_t> entries;
};

namespace {

void build_cells(htb_tree& t, int n_leaf) {
    struct Pending { int32_t level; int64_t b, e, parent; };
    std::vector<Pending> stack;
    stack.push_back({0, 0, t.n, -1});
    t.cell.reserve(static_cast<size_t>(2 * t.n + 1));
    while (!stack.empty()) {
        const Pending p = stack.back();
        stack.pop_back();
        const int64_t id = static_cast<int64_t>(t.cell.size());
        Cell c;
        c.level = p.level;
        c.begin = p.b;
        c.end = p.e;
        c.parent = p.parent;
        c.split = (p.e - p.b > n_leaf) && (p.level < kDeepest) ? 1 : 0;
        c.skip = 0;
        c.node = -1;
        t.cell.push_back(c);
        if (!c.split) continue;
        // children: runs of equal 3-bit digit below this level, found by bisection
        const int sh = 3 * (kDeepest - p.level - 1);
        int64_t bound[9];
        bound[0] = p.b;
        bound[8] = p.e;
        const uint64_t* kb = t.key.data();
        for (uint32_t d = 1; d < 8; ++d) {
            bound[d] = std::partition_point(kb + p.b, kb + p.e, [&](uint64_t k) {
                           return ((k >> sh) & 7u) < d;
                       }) - kb;
        }
        for (int d = 7; d >= 0; --d)
            if (bound[d + 1] > bound[d]) stack.push_back({p.level + 1, bound[d], bound[d + 1], id});
    }
    const int64_t nc = static_cast<int64_t>(t.cell.size());
    std::vector<int64_t> size(nc, 1);
    for (int64_t c = nc - 1; c > 0; --c) size[t.cell[c].parent] += size[c];
    for (int64_t c = 0; c < nc; ++c) t.cell[c].skip = c + size[c];
}

// Node sums, bottom-up: S = (sum m, sum m*x, sum m*v, sum m*a, sum m*jerk)
// starts from zero; a split node adds its children's S in key order (a
// single-particle child's S is 0 + its rounded products), an unsplit node its
// particles' rounded products in ascending order.  Children are one level
// deeper, so the nodes of one level depend only on the level below.
void node_sums(const htb_tree& t, int64_t q, const double* m, const double* x, const double* v, const double* a,
               const double* j, double* raw) {
    const int64_t ci = t.node_cell[q];
    const Cell& c = t.cell[ci];
    double s[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    auto products = [&](int64_t k, double* u) {   // u += the products of particle k
        const double mk = m[k];
        u[0] = u[0] + mk;
        for (int d = 0; d < 3; ++d) {
            u[1 + d] = u[1 + d] + mk * x[3 * k + d];
            u[4 + d] = u[4 + d] + mk * v[3 * k + d];
            u[7 + d] = u[7 + d] + mk * a[3 * k + d];
            u[10 + d] = u[10 + d] + mk * j[3 * k + d];
        }
    };
    if (c.split) {
        for (int64_t ch = ci + 1; ch < c.skip; ch = t.cell[ch].skip) {
            const Cell& cc = t.cell[ch];
            double u[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            if (cc.node >= 0) {
                for (int r = 0; r < 13; ++r) u[r] = raw[13 * cc.node + r];
            } else {
                products(cc.begin, u);
            }
            for (int r = 0; r < 13; ++r) s[r] = s[r] + u[r];
        }
    } else {
        for (int64_t k = c.begin; k < c.end; ++k) products(k, s);
    }
    for (int r = 0; r < 13; ++r) raw[13 * q + r] = s[r];
}

// Walk the pre-order cell array once for one group, without a stack.
void group_list(const htb_tree& t, int64_t gb, int64_t ge, const double lo[3], const double hi[3],
                double theta2, const double* s2_level, std::vector<int32_t>& out) {
    const int64_t nc = static_cast<int64_t>(t.cell.size());
    int64_t c = 0;
    while (c < nc) {
        const Cell& cl = t.cell[c];
        const bool overlaps = cl.begin < ge && gb < cl.end;
        bool open;
        if (overlaps) {
            open = true;
        } else if (cl.end - cl.begin == 1) {
            out.push_back(static_cast<int32_t>(cl.begin));
            c = cl.skip;
            continue;
        } else {
            const double* X = &t.nx[3 * cl.node];
            double gap[3];
            for (int d = 0; d < 3; ++d) gap[d] = std::max(std::max(lo[d] - X[d], X[d] - hi[d]), 0.0);
            const double d2 = (gap[0] * gap[0] + gap[1] * gap[1]) + gap[2] * gap[2];
            if (s2_level[cl.level] < theta2 * d2) {
                out.push_back(static_cast<int32_t>(t.n + cl.node));
                c = cl.skip;
                continue;
            }
            open = true;
        }
        if (open && cl.split) {
            c = c + 1;  // first child follows its parent in pre-order
        } else {
            for (int64_t k = cl.begin; k < cl.end; ++k) out.push_back(static_cast<int32_t>(k));
            c = cl.skip;
        }
    }
}

}  // namespace

namespace {
// Largest power of two h <= cap with t1 a multiple of h; 0 below 2^-40.
// t1 = m 2^(e-53) with m a 53-bit integer is a multiple of 2^j exactly when j
// is at most e - 53 + (trailing zero bits of m), so no trial division is needed.
double quantise(double cap, double t1) {
    if (!(cap > 0.0)) return 0.0;
    int e;
    std::frexp(cap, &e);
    int j = e - 1;  // 2^j <= cap < 2^(j+1)
    if (t1 != 0.0) {
        int et;
        const double mt = std::frexp(std::fabs(t1), &et);
        const uint64_t m = static_cast<uint64_t>(std::ldexp(mt, 53));
        j = std::min(j, et - 53 + __builtin_ctzll(m));
    }
    return j >= -40 ? std::ldexp(1.0, j) : 0.0;
}
inline double len3(const double* u) { return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

// Hermite corrector, Aarseth step and block quantisation for particle i
// (forces acc1, jerk1 at t1); returns 1 if the step fell below the floor.
inline int correct_one(int64_t i, double t1, double eta, double dt_tree, double* t0, double* dt, double* x, double* v,
                       double* a, double* jerk, const double* acc1, const double* jerk1) {
    const double D = t1 - t0[i];
    const double h2 = 0.5 * D, h3 = D / 3.0;
    double s2[3], s3[3], s2n[3];
    const double D2 = D * D, D3 = D2 * D, D4 = D2 * D2, D5 = D4 * D;
    for (int d = 0; d < 3; ++d) {
        const int64_t q = 3 * i + d;
        const double xp = x[q] + D * (v[q] + h2 * (a[q] + h3 * jerk[q]));
        const double vp = v[q] + D * (a[q] + h2 * jerk[q]);
        const double diff = a[q] - acc1[d];
        s2[d] = (-6.0 * diff - D * (4.0 * jerk[q] + 2.0 * jerk1[d])) / D2;  // a'' at t0
        s3[d] = (12.0 * diff + 6.0 * D * (jerk[q] + jerk1[d])) / D3;        // a'''
        x[q] = xp + s2[d] * (D4 / 24.0) + s3[d] * (D5 / 120.0);
        v[q] = vp + s2[d] * (D3 / 6.0) + s3[d] * (D4 / 24.0);
        a[q] = acc1[d];
        jerk[q] = jerk1[d];
        s2n[d] = s2[d] + D * s3[d];                                          // a'' at t1
    }
    const double na = len3(acc1), nj = len3(jerk1);
    const double n2 = len3(s2n), n3 = len3(s3);
    const double den = nj * n3 + n2 * n2;
    const double raw = den > 0.0 ? std::sqrt(eta * (na * n2 + nj * nj) / den) : dt_tree;
    const double h = quantise(std::min(std::min(raw, dt_tree), 2.0 * dt[i]), t1);
    t0[i] = t1;
    dt[i] = h;
    return h == 0.0 ? 1 : 0;
}

struct Row {  // ht_row layout
    int32_t idx, pad;
    double t0, m;
    double x[3], v[3], a[3], jerk[3];
};
static_assert(sizeof(Row) == 120, "update row layout");

}  // namespace

extern "C" {

int htb_hilbert_keys(int64_t n, const uint32_t* q, uint64_t* keys) {
    if (n < 0 || (n > 0 && (!q || !keys))) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) keys[i] = ph_key(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
    return 0;
}

int htb_build(htb_tree** out, int64_t n, const double* x, const double* v, const double* a,
              const double* jerk, const double* m, int32_t n_leaf, int32_t n_crit, double theta) {
    if (!out || n < 1 || n > INT32_MAX / 2 || !x || !v || !a || !jerk || !m || n_leaf < 1 || n_crit < 1 ||
        !(theta >= 0.0))
        return -1;
    htb_tree* t = new (std::nothrow) htb_tree();
    if (!t) return -3;
    try {
        t->n = n;
        // root cube
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = x[d];
        for (int64_t i = 1; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], x[3 * i + d]);
                hi[d] = std::max(hi[d], x[3 * i + d]);
            }
        double ext = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
        double side = 1.0;
        if (ext > 0.0) {
            int e;
            std::frexp(ext, &e);
            side = std::ldexp(1.0, e);
        }
        const double scale = std::ldexp(1.0, kAxisBits) / side;
        const double qmax = std::ldexp(1.0, kAxisBits) - 1.0;
        t->key.resize(n);
        t->perm.resize(n);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t q[3];
            for (int d = 0; d < 3; ++d) {
                double u = std::floor((x[3 * i + d] - lo[d]) * scale);
                u = std::min(std::max(u, 0.0), qmax);
                q[d] = static_cast<uint32_t>(u);
            }
            t->key[i] = ph_key(q[0], q[1], q[2]);
            t->perm[i] = i;
        }
        radix_sort(t->key, t->perm);
        // particles in the new order
        std::vector<double> sx(3 * n), sv(3 * n), sa(3 * n), sj(3 * n), sm(n);
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            const int64_t o = t->perm[k];
            sm[k] = m[o];
            for (int d = 0; d < 3; ++d) {
                sx[3 * k + d] = x[3 * o + d];
                sv[3 * k + d] = v[3 * o + d];
                sa[3 * k + d] = a[3 * o + d];
                sj[3 * k + d] = jerk[3 * o + d];
            }
        }
        build_cells(*t, n_leaf);
        const int64_t nc = static_cast<int64_t>(t->cell.size());
        int64_t M = 0;
        std::vector<int8_t> node_level;
        for (int64_t c = 0; c < nc; ++c)
            if (t->cell[c].end - t->cell[c].begin >= 2) {
                t->cell[c].node = M++;
                t->node_cell.push_back(c);
                node_level.push_back(static_cast<int8_t>(t->cell[c].level));
            }
        t->nm.resize(M);
        t->nx.resize(3 * M);
        t->nv.resize(3 * M);
        t->na.resize(3 * M);
        t->nj.resize(3 * M);
        {
            std::unique_ptr<double[]> raw(new double[static_cast<size_t>(13 * std::max<int64_t>(M, 1))]);
            std::vector<int64_t> at(kDeepest + 2, 0), by_level(static_cast<size_t>(M));
            for (int64_t k = 0; k < M; ++k) at[node_level[k] + 1]++;
            for (int l = 0; l <= kDeepest; ++l) at[l + 1] += at[l];
            std::vector<int64_t> fill(at.begin(), at.end() - 1);
            for (int64_t k = 0; k < M; ++k) by_level[fill[node_level[k]]++] = k;
            for (int l = kDeepest; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 256)
                for (int64_t r = at[l]; r < at[l + 1]; ++r)
                    node_sums(*t, by_level[r], sm.data(), sx.data(), sv.data(), sa.data(), sj.data(), raw.get());
            }
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < M; ++k) {
                const double* u = &raw[13 * k];
                t->nm[k] = u[0];
                for (int d = 0; d < 3; ++d) {
                    t->nx[3 * k + d] = u[1 + d] / u[0];
                    t->nv[3 * k + d] = u[4 + d] / u[0];
                    t->na[3 * k + d] = u[7 + d] / u[0];
                    t->nj[3 * k + d] = u[10 + d] / u[0];
                }
            }
        }
        // groups: first cell on each path with <= n_crit particles or no split
        for (int64_t c = 0; c < nc;) {
            const Cell& cl = t->cell[c];
            if (cl.end - cl.begin <= n_crit || !cl.split) {
                t->group_first.push_back(cl.begin);
                c = cl.skip;
            } else {
                c = c + 1;
            }
        }
        const int64_t G = static_cast<int64_t>(t->group_first.size());
        t->group_first.push_back(n);
        double s2_level[kDeepest + 1];
        for (int l = 0; l <= kDeepest; ++l) {
            const double s = std::ldexp(side, -l);
            s2_level[l] = s * s;
        }
        const double theta2 = theta * theta;
        std::vector<std::vector<int32_t>> lists(G);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t g = 0; g < G; ++g) {
            const int64_t gb = t->group_first[g], ge = t->group_first[g + 1];
            double blo[3], bhi[3];
            for (int d = 0; d < 3; ++d) blo[d] = bhi[d] = sx[3 * gb + d];
            for (int64_t k = gb + 1; k < ge; ++k)
                for (int d = 0; d < 3; ++d) {
                    blo[d] = std::min(blo[d], sx[3 * k + d]);
                    bhi[d] = std::max(bhi[d], sx[3 * k + d]);
                }
            group_list(*t, gb, ge, blo, bhi, theta2, s2_level, lists[g]);
        }
        t->list_off.resize(G + 1);
        t->list_off[0] = 0;
        for (int64_t g = 0; g < G; ++g) t->list_off[g + 1] = t->list_off[g] + static_cast<int64_t>(lists[g].size());
        t->entries.resize(t->list_off[G]);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t g = 0; g < G; ++g)
            if (!lists[g].empty())
                std::memcpy(&t->entries[t->list_off[g]], lists[g].data(), lists[g].size() * sizeof(int32_t));
    } catch (const std::bad_alloc&) {
        delete t;
        return -3;
    }
    *out = t;
    return 0;
}

int htb_sizes(const htb_tree* t, int64_t* n_node, int64_t* n_group, int64_t* n_entries) {
    if (!t) return -1;
    if (n_node) *n_node = static_cast<int64_t>(t->nm.size());
    if (n_group) *n_group = static_cast<int64_t>(t->group_first.size()) - 1;
    if (n_entries) *n_entries = static_cast<int64_t>(t->entries.size());
    return 0;
}

int htb_get(const htb_tree* t, int64_t* perm, uint64_t* keys, double* node_m, double* node_x, double* node_v,
            double* node_a, double* node_j, int32_t* node_level, int64_t* node_begin, int64_t* node_end,
            int64_t* group_first, int64_t* list_off, int32_t* entries) {
    if (!t) return -1;
    const size_t M = t->nm.size();
    auto put = [](auto* dst, const auto& src) {
        if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(src[0]));
    };
    put(perm, t->perm);
    put(keys, t->key);
    put(node_m, t->nm);
    put(node_x, t->nx);
    put(node_v, t->nv);
    put(node_a, t->na);
    put(node_j, t->nj);
    for (size_t k = 0; k < M; ++k) {
        const Cell& c = t->cell[t->node_cell[k]];
        if (node_level) node_level[k] = c.level;
        if (node_begin) node_begin[k] = c.begin;
        if (node_end) node_end[k] = c.end;
    }
    put(group_first, t->group_first);
    put(list_off, t->list_off);
    put(entries, t->entries);
    return 0;
}

void htb_free(htb_tree* t) { delete t; }

int htb_next_block(int64_t n, const double* t0, const double* dt, double* t_next, int32_t* active,
                   int64_t* n_active) {
    if (n < 1 || !t0 || !dt || !t_next || !active || !n_active) return -1;
    double tmin = std::numeric_limits<double>::infinity();
#pragma omp parallel for reduction(min : tmin) schedule(static)
    for (int64_t i = 0; i < n; ++i) tmin = std::min(tmin, t0[i] + dt[i]);
    const int nth = omp_get_max_threads();
    std::vector<int64_t> count(nth + 1, 0);
#pragma omp parallel num_threads(nth)
    {
        const int id = omp_get_thread_num(), nt = omp_get_num_threads();
        const int64_t b = n * id / nt, e = n * (id + 1) / nt;
        int64_t c = 0;
        for (int64_t i = b; i < e; ++i) c += (t0[i] + dt[i] == tmin);
        count[id + 1] = c;
#pragma omp barrier
#pragma omp single
        for (int k = 0; k < nt; ++k) count[k + 1] += count[k];
        int64_t p = count[id];
        for (int64_t i = b; i < e; ++i)
            if (t0[i] + dt[i] == tmin) active[p++] = static_cast<int32_t>(i);
    }
    *t_next = tmin;
    *n_active = count[nth];
    return 0;
}


int htb_correct(int64_t n_active, const int32_t* ids, double t1, double eta, double dt_tree, double* t0,
                double* dt, double* x, double* v, double* a, double* jerk, const double* acc1,
                const double* jerk1) {
    if (n_active < 0 || (n_active > 0 && (!ids || !t0 || !dt || !x || !v || !a || !jerk || !acc1 || !jerk1)))
        return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < n_active; ++k)
        bad |= correct_one(ids[k], t1, eta, dt_tree, t0, dt, x, v, a, jerk, acc1 + 3 * k, jerk1 + 3 * k);
    return bad ? -2 : 0;
}

int htb_initial_steps(int64_t n, double eta, double dt_tree, const double* a, const double* jerk, double* dt) {
    if (n < 0 || (n > 0 && (!a || !jerk || !dt))) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        const double na = len3(&a[3 * i]), nj = len3(&jerk[3 * i]);
        const double raw = nj > 0.0 ? eta * na / nj : dt_tree;
        dt[i] = quantise(std::min(raw, dt_tree), 0.0);
        if (dt[i] == 0.0) bad = 1;
    }
    return bad ? -2 : 0;
}

int htb_next_block_many(int32_t n_clusters, htb_cluster* cl) {
    if (n_clusters < 0 || (n_clusters > 0 && !cl)) return -1;
    for (int32_t k = 0; k < n_clusters; ++k)
        if (cl[k].n < 1 || !cl[k].t0 || !cl[k].dt || !cl[k].active) return -1;
    // Chunks of at most kChunk particles, so that the largest cluster does not
    // set the time.  One parallel pass: each chunk finds its earliest next time
    // and lists its particles due then, in its own slice of the cluster's
    // active array.  Then, per cluster, t_next is the earliest over its chunks
    // and the lists of the chunks due at t_next are moved down, in order.
    constexpr int64_t kChunk = 8192;
    struct Chunk {
        int32_t k;
        int64_t b, e;
        double tmin;
        int64_t cnt;
    };
    std::vector<Chunk> ch;
    for (int32_t k = 0; k < n_clusters; ++k)
        for (int64_t b = 0; b < cl[k].n; b += kChunk) ch.push_back(Chunk{k, b, std::min(cl[k].n, b + kChunk), 0.0, 0});
    const int64_t nch = static_cast<int64_t>(ch.size());
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t q = 0; q < nch; ++q) {
        Chunk& h = ch[q];
        const htb_cluster& c = cl[h.k];
        double tmin = std::numeric_limits<double>::infinity();
        int32_t* out = c.active + h.b;
        int64_t cnt = 0;
        for (int64_t i = h.b; i < h.e; ++i) {
            const double t = c.t0[i] + c.dt[i];
            if (t < tmin) {
                tmin = t;
                cnt = 0;
            }
            if (t == tmin) out[cnt++] = static_cast<int32_t>(i);
        }
        h.tmin = tmin;
        h.cnt = cnt;
    }
    for (int32_t k = 0; k < n_clusters; ++k) {
        cl[k].t_next = std::numeric_limits<double>::infinity();
        cl[k].n_active = 0;
    }
    for (const Chunk& h : ch) cl[h.k].t_next = std::min(cl[h.k].t_next, h.tmin);
    for (const Chunk& h : ch) {   // chunks in ascending order, destinations never pass their sources
        htb_cluster& c = cl[h.k];
        if (h.tmin != c.t_next) continue;
        if (c.n_active != h.b) std::memmove(c.active + c.n_active, c.active + h.b, static_cast<size_t>(h.cnt) * 4);
        c.n_active += h.cnt;
    }
    return 0;
}

int htb_correct_many(int32_t n_clusters, htb_cluster* cl, const int64_t* off, const double* acc, const double* jerk,
                     const double* pot, const int64_t* row_off, void* rows, int32_t* rebuild) {
    if (n_clusters < 0 || (n_clusters > 0 && (!cl || !off || !acc || !jerk || !pot || !row_off || !rows || !rebuild)))
        return -1;
    // One flat loop over every active particle of every cluster (clusters differ
    // in size by orders of magnitude, so a loop over clusters would leave one
    // thread with the largest); first[k] is cluster k's first flat index.
    std::vector<int64_t> first(static_cast<size_t>(n_clusters) + 1, 0);
    for (int32_t k = 0; k < n_clusters; ++k) {
        first[k + 1] = first[k] + cl[k].n_active;
        rebuild[k] = std::fmod(cl[k].t_next, cl[k].dt_tree) == 0.0 ? 1 : 0;
    }
    const int64_t total = first[n_clusters];
    int bad = 0;
#pragma omp parallel for schedule(static, 256) reduction(| : bad)
    for (int64_t f = 0; f < total; ++f) {
        const int32_t k = static_cast<int32_t>(std::upper_bound(first.begin(), first.end(), f) - first.begin()) - 1;
        htb_cluster& c = cl[k];
        const int64_t q = f - first[k], o = off[k] + q;
        const int32_t i = c.active[q];
        bad |= correct_one(i, c.t_next, c.eta, c.dt_tree, c.t0, c.dt, c.x, c.v, c.a, c.jerk, acc + 3 * o, jerk + 3 * o);
        c.pot[i] = pot[o];
        if (rebuild[k]) continue;
        Row& w = static_cast<Row*>(rows)[row_off[k] + q];
        w.idx = i;
        w.pad = 0;
        w.t0 = c.t0[i];
        w.m = c.m[i];
        for (int d = 0; d < 3; ++d) {
            w.x[d] = c.x[3 * i + d];
            w.v[d] = c.v[3 * i + d];
            w.a[d] = c.a[3 * i + d];
            w.jerk[d] = c.jerk[3 * i + d];
        }
    }
    return bad ? -2 : 0;
}

}  // extern "C"
