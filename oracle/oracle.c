/*
 * FP64 CPU oracle for the Barnes-Hut hot path of "On Distributed Gravitational
 * N-Body Simulations" (Brandt, arXiv:2203.08966).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the GPU library: every step below
 * is written out again, plainly, from the paper.
 *
 * Every function is slow and straightforward on purpose: no blocking, fusion
 * or reordering beyond what the definition states.  Per-target loops run under
 * OpenMP; that changes no arithmetic, because each target is independent.
 *
 * Compile with -ffp-contract=off: the key quantisation must round exactly as
 * written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#pragma STDC FP_CONTRACT OFF

#define ORC_LEVELS 21 /* bits per dimension of a spatial key (Sec. 4.4) */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Direct summation (Sec. 2.1, equation of motion with G = 1 and the softened
 * separation (|r_i - r_j|^2 + eps^2)^(1/2); potential as the superposition of
 * point-mass potentials, Sec. 2.2).  Self-pair skipped by index.
 * acc[t] and phi[t] are written for body targets[t].
 * ---------------------------------------------------------------------- */
void orc_direct(int64_t n, const double *pos, const double *mass, double eps,
                int64_t nt, const int64_t *targets, double *acc, double *phi)
{
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets[t];
        double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double dx = pos[3 * j + 0] - pos[3 * i + 0];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            double s2 = dx * dx + dy * dy + dz * dz + e2;
            double s = sqrt(s2);
            double f = mass[j] / (s2 * s);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
            p -= mass[j] / s;
        }
        acc[3 * t + 0] = ax;
        acc[3 * t + 1] = ay;
        acc[3 * t + 2] = az;
        if (phi)
            phi[t] = p;
    }
}

/* ------------------------------------------------------------------------
 * Root cell (Sec. 3: the root is the bounding box of all bodies; Sec. 4.4 maps
 * coordinates onto [0, 2^21)).  Reading: the root is a cube whose side L is
 * the smallest power of two such that, with the lower corner snapped down to
 * a multiple of L/2, every body lies strictly inside it.
 * ---------------------------------------------------------------------- */
void orc_root_cube(int64_t n, const double *pos, double *lo, double *Lout)
{
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d)
        mn[d] = mx[d] = pos[d];
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * i + d];
            if (v < mn[d]) mn[d] = v;
            if (v > mx[d]) mx[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d)
        if (mx[d] - mn[d] > ext)
            ext = mx[d] - mn[d];
    double L = 1.0;
    if (ext > 0.0) {
        int e;
        frexp(ext, &e); /* 2^(e-1) <= ext < 2^e */
        L = ldexp(1.0, e - 1);
    }
    for (;;) {
        double half = 0.5 * L;
        int ok = 1;
        for (int d = 0; d < 3; ++d) {
            lo[d] = floor(mn[d] / half) * half;
            if (!(mx[d] < lo[d] + L))
                ok = 0;
        }
        if (ok)
            break;
        L *= 2.0;
    }
    *Lout = L;
}

/* ------------------------------------------------------------------------
 * Morton key (Sec. 4.4): interleave the 21-bit integer coordinates one bit at
 * a time, most significant first, with x more significant than y than z
 * (the octant labels of the hashed-octree figure, Sec. 4.7).  Written as the
 * plain bit loop.
 * ---------------------------------------------------------------------- */
uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t key = 0;
    for (int b = ORC_LEVELS - 1; b >= 0; --b) {
        key = (key << 3) | ((uint64_t)((qx >> b) & 1u) << 2) |
              ((uint64_t)((qy >> b) & 1u) << 1) | (uint64_t)((qz >> b) & 1u);
    }
    return key;
}

/* Quantise one coordinate onto [0, 2^21 - 1]: floor((x - lo) * 2^21 / L). */
static uint32_t quantise(double x, double lo, double scale)
{
    double t = (x - lo) * scale;
    double f = floor(t);
    if (f < 0.0)
        f = 0.0;
    if (f > (double)((1u << ORC_LEVELS) - 1u))
        f = (double)((1u << ORC_LEVELS) - 1u);
    return (uint32_t)f;
}

void orc_keys(int64_t n, const double *pos, const double *lo, double L, uint64_t *keys)
{
    const double scale = ldexp(1.0, ORC_LEVELS) / L;
    for (int64_t i = 0; i < n; ++i)
        keys[i] = orc_interleave(quantise(pos[3 * i + 0], lo[0], scale),
                                 quantise(pos[3 * i + 1], lo[1], scale),
                                 quantise(pos[3 * i + 2], lo[2], scale));
}

/* ------------------------------------------------------------------------
 * Sort bodies by key (Sec. 4.4); ties keep the original index order.
 * perm[r] = original index of the body at sorted rank r.
 * ---------------------------------------------------------------------- */
static const uint64_t *g_sort_keys;

static int cmp_rank(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki != kj)
        return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

void orc_sort(int64_t n, const uint64_t *keys, int64_t *perm)
{
    for (int64_t i = 0; i < n; ++i)
        perm[i] = i;
    g_sort_keys = keys;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_rank);
    g_sort_keys = NULL;
}

/* ------------------------------------------------------------------------
 * Octree (Sec. 3, Barnes-Hut loop body: build tree; nodes carry the 8-bit
 * child mask and are serialised in pre-order, Sec. 4.2; cell keys are the
 * hashed-octree keys 1<<3k | prefix, Sec. 4.7).
 *
 * Reading for a leaf capacity B: a cell is split in half in each dimension
 * when it holds more than B bodies and is above the finest key level 21;
 * only non-empty children are created.  B = 1 is the paper's tree.  Bodies at
 * level 21 that share a key stay together in one leaf.
 *
 * Written top-down and recursively, straight from that definition, over the
 * key-sorted bodies.  Nodes come out in pre-order.  With NULL output arrays
 * only the node count is returned.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t m;
    uint64_t *hkey;
    int32_t *level, *begin, *count, *next, *parent, *cmask;
} tree_out;

static void split_cell(tree_out *t, const uint64_t *keys, int B, int k,
                       uint64_t prefix, int64_t b, int64_t e, int64_t parent)
{
    const int64_t id = t->m++;
    const int w = t->hkey != NULL;
    if (w) {
        t->hkey[id] = ((uint64_t)1 << (3 * k)) | prefix;
        t->level[id] = k;
        t->begin[id] = (int32_t)b;
        t->count[id] = (int32_t)(e - b);
        t->parent[id] = (int32_t)parent;
        t->cmask[id] = 0;
    }
    if (e - b > B && k < ORC_LEVELS) {
        const int shift = 3 * (ORC_LEVELS - (k + 1));
        int64_t s = b;
        while (s < e) {
            const unsigned d = (unsigned)((keys[s] >> shift) & 7u);
            int64_t f = s;
            while (f < e && (unsigned)((keys[f] >> shift) & 7u) == d)
                ++f;
            if (w)
                t->cmask[id] |= 1 << d;
            split_cell(t, keys, B, k + 1, (prefix << 3) | d, s, f, id);
            s = f;
        }
    }
    if (w)
        t->next[id] = (int32_t)t->m;
}

int64_t orc_build(int64_t n, const uint64_t *sorted_keys, int leaf_size, uint64_t *hkey,
                  int32_t *level, int32_t *begin, int32_t *count, int32_t *next,
                  int32_t *parent, int32_t *cmask)
{
    tree_out t = {0, hkey, level, begin, count, next, parent, cmask};
    split_cell(&t, sorted_keys, leaf_size, 0, 0, 0, n, -1);
    return t.m;
}

/* ------------------------------------------------------------------------
 * Cell moments (Sec. 2.2, truncated multipole expansion): total mass M0,
 * centre of mass (the dipole vanishes about it; the COM is the mass-weighted
 * mean position -- the displayed COM formula omits the division by the
 * mass), and Q_ab = sum m (3 y_a y_b - |y|^2 delta_ab) with y the body's
 * offset from the COM.  Computed per cell directly from its bodies.
 * A massless cell gets its geometric centre as COM and Q = 0.
 * Q layout: xx, xy, xz, yy, yz, zz.
 * ---------------------------------------------------------------------- */
void orc_moments(int64_t m, const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                 const int32_t *count, const double *spos, const double *smass,
                 const double *lo, double L, double *M, double *com, double *Q)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < m; ++c) {
        const int64_t b = begin[c], e = b + count[c];
        double mt = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t j = b; j < e; ++j) {
            mt += smass[j];
            sx += smass[j] * spos[3 * j + 0];
            sy += smass[j] * spos[3 * j + 1];
            sz += smass[j] * spos[3 * j + 2];
        }
        double cx, cy, cz;
        if (mt > 0.0) {
            cx = sx / mt;
            cy = sy / mt;
            cz = sz / mt;
        } else {
            /* geometric centre of the cell from its hashed key */
            const int k = level[c];
            const uint64_t prefix = hkey[c] ^ ((uint64_t)1 << (3 * k));
            uint32_t ix = 0, iy = 0, iz = 0;
            for (int l = 0; l < k; ++l) {
                unsigned d = (unsigned)((prefix >> (3 * (k - 1 - l))) & 7u);
                ix = (ix << 1) | ((d >> 2) & 1u);
                iy = (iy << 1) | ((d >> 1) & 1u);
                iz = (iz << 1) | (d & 1u);
            }
            const double side = ldexp(L, -k);
            cx = lo[0] + (ix + 0.5) * side;
            cy = lo[1] + (iy + 0.5) * side;
            cz = lo[2] + (iz + 0.5) * side;
        }
        double q[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = b; j < e; ++j) {
            const double y0 = spos[3 * j + 0] - cx;
            const double y1 = spos[3 * j + 1] - cy;
            const double y2 = spos[3 * j + 2] - cz;
            const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
            const double mj = smass[j];
            q[0] += mj * (3.0 * y0 * y0 - r2);
            q[1] += mj * (3.0 * y0 * y1);
            q[2] += mj * (3.0 * y0 * y2);
            q[3] += mj * (3.0 * y1 * y1 - r2);
            q[4] += mj * (3.0 * y1 * y2);
            q[5] += mj * (3.0 * y2 * y2 - r2);
        }
        M[c] = mt;
        com[3 * c + 0] = cx;
        com[3 * c + 1] = cy;
        com[3 * c + 2] = cz;
        for (int a = 0; a < 6; ++a)
            Q[6 * c + a] = q[a];
    }
}

/* ------------------------------------------------------------------------
 * Tree walk (Sec. 3, "Compute Cell Force" of the Barnes-Hut loop body).
 *
 * For body i, start at the root and, for each child C of the current node in
 * octant order:
 *   - C holds one body            -> particle-particle (skipped if it is i);
 *   - side/distance < theta       -> particle-cell with C's expansion
 *                                    (tested as side^2 < theta^2 * d^2, d from
 *                                    body i to C's centre of mass);
 *   - C is a leaf holding several -> particle-particle with each of its
 *     bodies (the reading for a leaf capacity above one);
 *   - otherwise                   -> recurse into C.
 * A root that is itself a leaf interacts particle-particle with all its
 * bodies.  Softening applies to every term.  order 0 uses the monopole only
 * (the original method); order 2 adds the quadrupole of the truncated
 * expansion, whose field is  a = Q x / s^5 - (5/2)(x.Q.x) x / s^7,  with
 * potential -(x.Q.x)/(2 s^5), x = r_i - COM, s^2 = |x|^2 + eps^2.
 *
 * Results per target t (a sorted-order body index): acc, phi, the counts of
 * particle-particle and particle-cell interactions, the number of bodies
 * those interactions stand for (p-p counts one, p-c the cell's count), and a
 * flag set when any
 * acceptance test of this body was within a relative 1e-5 of its threshold
 * (|side^2 - theta^2 d^2| < 1e-5 side^2), where a reduced-precision evaluation
 * may legitimately decide the other way.
 * ---------------------------------------------------------------------- */
typedef struct {
    const int32_t *level, *begin, *count, *next;
    const double *M, *com, *Q;
    const double *spos, *smass;
    double L, theta2, e2;
    int order;
} walk_ctx;

typedef struct {
    double a[3], phi;
    int64_t npp, npc, ncov;
    int flag;
} walk_acc;

static void pp(const walk_ctx *w, int64_t i, int64_t j, walk_acc *r)
{
    const double dx = w->spos[3 * j + 0] - w->spos[3 * i + 0];
    const double dy = w->spos[3 * j + 1] - w->spos[3 * i + 1];
    const double dz = w->spos[3 * j + 2] - w->spos[3 * i + 2];
    const double s2 = dx * dx + dy * dy + dz * dz + w->e2;
    const double s = sqrt(s2);
    const double f = w->smass[j] / (s2 * s);
    r->a[0] += f * dx;
    r->a[1] += f * dy;
    r->a[2] += f * dz;
    r->phi -= w->smass[j] / s;
    r->npp += 1;
    r->ncov += 1;
}

static void pc(const walk_ctx *w, int64_t i, int64_t c, const double x[3], double d2, walk_acc *r)
{
    const double Mc = w->M[c];
    const double s2 = d2 + w->e2;
    const double s = sqrt(s2);
    const double inv = 1.0 / s;
    const double inv2 = inv * inv;
    const double inv3 = inv2 * inv;
    r->a[0] -= Mc * x[0] * inv3;
    r->a[1] -= Mc * x[1] * inv3;
    r->a[2] -= Mc * x[2] * inv3;
    r->phi -= Mc * inv;
    if (w->order >= 2) {
        const double *q = &w->Q[6 * c];
        const double qx = q[0] * x[0] + q[1] * x[1] + q[2] * x[2];
        const double qy = q[1] * x[0] + q[3] * x[1] + q[4] * x[2];
        const double qz = q[2] * x[0] + q[4] * x[1] + q[5] * x[2];
        const double xqx = x[0] * qx + x[1] * qy + x[2] * qz;
        const double inv5 = inv3 * inv2;
        const double inv7 = inv5 * inv2;
        r->a[0] += qx * inv5 - 2.5 * xqx * x[0] * inv7;
        r->a[1] += qy * inv5 - 2.5 * xqx * x[1] * inv7;
        r->a[2] += qz * inv5 - 2.5 * xqx * x[2] * inv7;
        r->phi -= 0.5 * xqx * inv5;
    }
    (void)i;
    r->npc += 1;
    r->ncov += w->count[c];
}

static void leaf_pp(const walk_ctx *w, int64_t i, int64_t c, walk_acc *r)
{
    const int64_t b = w->begin[c], e = b + w->count[c];
    for (int64_t j = b; j < e; ++j)
        if (j != i)
            pp(w, i, j, r);
}

static void cell_force(const walk_ctx *w, int64_t node, int64_t i, walk_acc *r)
{
    for (int64_t c = node + 1; c < w->next[node]; c = w->next[c]) {
        if (w->count[c] == 1) {
            if (w->begin[c] != i)
                pp(w, i, w->begin[c], r);
            continue;
        }
        const double side = ldexp(w->L, -w->level[c]);
        double x[3];
        for (int d = 0; d < 3; ++d)
            x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
        const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double lhs = side * side, rhs = w->theta2 * d2;
        if (fabs(lhs - rhs) < 1e-5 * lhs)
            r->flag = 1;
        if (lhs < rhs)
            pc(w, i, c, x, d2, r);
        else if (w->next[c] == c + 1)
            leaf_pp(w, i, c, r);
        else
            cell_force(w, c, i, r);
    }
}

void orc_walk(int64_t m, const int32_t *level, const int32_t *begin, const int32_t *count,
              const int32_t *next, const double *M, const double *com, const double *Q,
              const double *spos, const double *smass, double L, double theta, double eps,
              int order, int64_t nt, const int64_t *targets, double *acc, double *phi,
              int64_t *npp, int64_t *npc, int64_t *ncov, int32_t *flag)
{
    walk_ctx w = {level, begin, count, next, M, com, Q, spos, smass,
                  L, theta * theta, eps * eps, order};
    (void)m;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets[t];
        walk_acc r;
        memset(&r, 0, sizeof(r));
        if (next[0] == 1)
            leaf_pp(&w, i, 0, &r); /* the root is a leaf */
        else
            cell_force(&w, 0, i, &r);
        for (int d = 0; d < 3; ++d)
            acc[3 * t + d] = r.a[d];
        if (phi) phi[t] = r.phi;
        if (npp) npp[t] = r.npp;
        if (npc) npc[t] = r.npc;
        if (ncov) ncov[t] = r.ncov;
        if (flag) flag[t] = r.flag;
    }
}

/* ========================================================================
 * Learned acceptance criterion.
 *
 * Features of a (body, cell) pair, all scale-free (x = body - COM, d = |x|,
 * n = x/d, g = COM - cell centre, l = cell side, Q the traceless quadrupole):
 *   f0 l/d            f1 (l/d)^2          f2 |g|/l        f3 n.g/l
 *   f4 distance from the body to the cell's cube / d (0 inside)
 *   f5 n.Q.n/(M l^2)  f6 |Q|_F/(M l^2)    f7 log2(count)/21
 *   f8 eps/d          f9 1 if the cell is a leaf
 * Label: log10 of |a_pc - a_exact| / |a_exact|, the error of the cell's
 * particle-cell term (order 2) relative to the cell's exact contribution
 * (direct sum over its bodies), floored at 1e-12.
 * ====================================================================== */

/* cell centre from the hashed key */
static void cell_centre(uint64_t hkey, int k, const double *lo, double L, double c[3])
{
    const uint64_t prefix = hkey ^ ((uint64_t)1 << (3 * k));
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int l = 0; l < k; ++l) {
        unsigned d = (unsigned)((prefix >> (3 * (k - 1 - l))) & 7u);
        ix = (ix << 1) | ((d >> 2) & 1u);
        iy = (iy << 1) | ((d >> 1) & 1u);
        iz = (iz << 1) | (d & 1u);
    }
    const double side = ldexp(L, -k);
    c[0] = lo[0] + (ix + 0.5) * side;
    c[1] = lo[1] + (iy + 0.5) * side;
    c[2] = lo[2] + (iz + 0.5) * side;
}

void orc_mac_features(const double *r, const double *centre, double side, const double *com,
                      double M, const double *Q, int count, int is_leaf, double eps, double *f)
{
    double x[3], g[3], n[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = r[a] - com[a];
        g[a] = com[a] - centre[a];
    }
    const double d = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int a = 0; a < 3; ++a)
        n[a] = x[a] / d;
    f[0] = side / d;
    f[1] = f[0] * f[0];
    f[2] = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) / side;
    f[3] = (n[0] * g[0] + n[1] * g[1] + n[2] * g[2]) / side;
    double db2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double t = fabs(r[a] - centre[a]) - 0.5 * side;
        if (t > 0.0)
            db2 += t * t;
    }
    f[4] = sqrt(db2) / d;
    /* full symmetric Q from xx xy xz yy yz zz */
    const double q[3][3] = {{Q[0], Q[1], Q[2]}, {Q[1], Q[3], Q[4]}, {Q[2], Q[4], Q[5]}};
    double nqn = 0.0, qf = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            nqn += n[a] * q[a][b] * n[b];
            qf += q[a][b] * q[a][b];
        }
    const double ml2 = M * side * side;
    f[5] = ml2 > 0.0 ? nqn / ml2 : 0.0;
    f[6] = ml2 > 0.0 ? sqrt(qf) / ml2 : 0.0;
    f[7] = log2((double)count) / 21.0;
    f[8] = eps / d;
    f[9] = is_leaf ? 1.0 : 0.0;
}

/* SplitMix64 (Steele, Lea & Flood 2014): the finaliser applied to x. */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* keep a candidate (body rank i, node c) with probability p */
static int keep_pair(uint64_t seed, int64_t i, int64_t c, double p)
{
    const uint64_t h = orc_splitmix64(seed ^ (((uint64_t)i << 32) | (uint64_t)(uint32_t)c));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0) < p;
}

static int inside_cell(const double *r, const double *centre, double side)
{
    for (int a = 0; a < 3; ++a)
        if (fabs(r[a] - centre[a]) > 0.5 * side)
            return 0;
    return 1;
}

/* round to bfloat16, nearest even */
static double bf16r(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* The network as the bf16 inference evaluates it (see oracle/mlp.py):
 * parameters W1[32][10] b1[32] W2[32][32] b2[32] w3[32] b3. */
double orc_mlp_bf16(const double *p, const double *f)
{
    const double *W1 = p, *b1 = p + 320, *W2 = p + 352, *b2 = p + 1376, *w3 = p + 1408;
    const double b3 = (double)(float)p[1440];
    double h1[32], out = 0.0;
    for (int u = 0; u < 32; ++u) {
        double s = bf16r(b1[u]);
        for (int k = 0; k < 10; ++k)
            s += bf16r(W1[u * 10 + k]) * bf16r(f[k]);
        h1[u] = bf16r(s > 0.0 ? s : 0.0);
    }
    for (int u = 0; u < 32; ++u) {
        double s = (double)(float)b2[u];
        for (int k = 0; k < 32; ++k)
            s += bf16r(W2[u * 32 + k]) * h1[k];
        if (s > 0.0)
            out += (double)(float)w3[u] * s;
    }
    return out + b3;
}

typedef struct {
    walk_ctx w;
    const uint64_t *hkey;
    const double *lo;
    double tlo2, thi2, eps;
    /* samples */
    uint64_t seed;
    double keep;
    int64_t cap, slot0, n_cand;
    double *feat, *label;
    int32_t *node;
    /* learned decision */
    const double *mlp;
    double log10tau;
} mac_ctx;

static void cell_label(const mac_ctx *m, int64_t i, int64_t c, double *lab)
{
    const walk_ctx *w = &m->w;
    walk_acc ex, ap;
    memset(&ex, 0, sizeof(ex));
    memset(&ap, 0, sizeof(ap));
    leaf_pp(w, i, c, &ex);
    double x[3];
    for (int d = 0; d < 3; ++d)
        x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
    pc(w, i, c, x, x[0] * x[0] + x[1] * x[1] + x[2] * x[2], &ap);
    const double e0 = ap.a[0] - ex.a[0], e1 = ap.a[1] - ex.a[1], e2 = ap.a[2] - ex.a[2];
    const double ne = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    const double na = sqrt(ex.a[0] * ex.a[0] + ex.a[1] * ex.a[1] + ex.a[2] * ex.a[2]);
    double rel = na > 0.0 ? ne / na : 1e-12;
    if (rel < 1e-12)
        rel = 1e-12;
    *lab = log10(rel);
}

static void pair_features(const mac_ctx *m, int64_t i, int64_t c, double *f)
{
    const walk_ctx *w = &m->w;
    double centre[3];
    cell_centre(m->hkey[c], w->level[c], m->lo, w->L, centre);
    orc_mac_features(&w->spos[3 * i], centre, ldexp(w->L, -w->level[c]), &w->com[3 * c],
                     w->M[c], &w->Q[6 * c], w->count[c], w->next[c] == c + 1, m->eps, f);
}

/* Candidates of body i: walk at theta_lo (everything at or above theta_lo
 * is opened); every multi-body cell with theta_lo <= l/d < theta_hi that
 * does not contain the body is a candidate; candidates kept by the hash. */
static void sample_walk(mac_ctx *m, int64_t node, int64_t i, int64_t *k)
{
    const walk_ctx *w = &m->w;
    for (int64_t c = node + 1; c < w->next[node]; c = w->next[c]) {
        if (w->count[c] == 1)
            continue;
        const double side = ldexp(w->L, -w->level[c]);
        double x[3];
        for (int d = 0; d < 3; ++d)
            x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
        const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double s2 = side * side;
        if (s2 < m->tlo2 * d2)
            continue; /* accepted below the band */
        if (s2 < m->thi2 * d2) {
            double centre[3];
            cell_centre(m->hkey[c], w->level[c], m->lo, w->L, centre);
            if (!inside_cell(&w->spos[3 * i], centre, side)) {
                m->n_cand++;
                if (keep_pair(m->seed, i, c, m->keep) && *k < m->cap) {
                    const int64_t o = m->slot0 + *k;
                    pair_features(m, i, c, &m->feat[10 * o]);
                    cell_label(m, i, c, &m->label[o]);
                    m->node[o] = (int32_t)c;
                    ++*k;
                }
            }
        }
        if (w->next[c] != c + 1)
            sample_walk(m, c, i, k);
    }
}

/* Per target rank t (targets are sorted ranks): up to cap kept candidates in
 * pre-order at slot t*cap.. of feat (10 each), label, node; count[t]. */
void orc_mac_samples(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                     const int32_t *count, const int32_t *next, const double *M,
                     const double *com, const double *Q, const double *spos,
                     const double *smass, const double *lo, double L, double eps,
                     double theta_lo, double theta_hi, double keep, uint64_t seed, int64_t nt,
                     const int64_t *targets, int64_t cap, double *feat, double *label,
                     int32_t *node, int64_t *cnt)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; ++t) {
        mac_ctx m;
        memset(&m, 0, sizeof(m));
        m.w = (walk_ctx){level, begin, count, next, M, com, Q, spos, smass, L, 0.0, eps * eps, 2};
        m.hkey = hkey;
        m.lo = lo;
        m.tlo2 = theta_lo * theta_lo;
        m.thi2 = theta_hi * theta_hi;
        m.eps = eps;
        m.seed = seed;
        m.keep = keep;
        m.cap = cap;
        m.slot0 = cap * t;
        m.feat = feat;
        m.label = label;
        m.node = node;
        int64_t k = 0;
        if (next[0] != 1)
            sample_walk(&m, 0, targets[t], &k);
        cnt[t] = k;
    }
}

/* Tree walk with the learned criterion: below theta_lo accept, at or above
 * theta_hi or with the body inside the cell open, otherwise accept iff the
 * network's predicted log10 relative error is below log10tau.  The flag also
 * marks decisions within 1e-3 of log10tau and bodies within 1e-6 side of a
 * cell face, where a reduced-precision evaluation may decide the other way. */
static void cell_force_mlp(mac_ctx *m, int64_t node, int64_t i, walk_acc *r)
{
    const walk_ctx *w = &m->w;
    for (int64_t c = node + 1; c < w->next[node]; c = w->next[c]) {
        if (w->count[c] == 1) {
            if (w->begin[c] != i)
                pp(w, i, w->begin[c], r);
            continue;
        }
        const double side = ldexp(w->L, -w->level[c]);
        double x[3];
        for (int d = 0; d < 3; ++d)
            x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
        const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double s2 = side * side;
        int accept;
        if (fabs(s2 - m->tlo2 * d2) < 1e-5 * s2 || fabs(s2 - m->thi2 * d2) < 1e-5 * s2)
            r->flag = 1;
        if (s2 < m->tlo2 * d2) {
            accept = 1;
        } else if (s2 >= m->thi2 * d2) {
            accept = 0;
        } else {
            double centre[3];
            cell_centre(m->hkey[c], w->level[c], m->lo, w->L, centre);
            int in = inside_cell(&w->spos[3 * i], centre, side);
            for (int a = 0; a < 3; ++a)
                if (fabs(fabs(w->spos[3 * i + a] - centre[a]) - 0.5 * side) < 1e-6 * side)
                    r->flag = 1;
            if (in) {
                accept = 0;
            } else {
                double f[10];
                pair_features(m, i, c, f);
                const double pred = orc_mlp_bf16(m->mlp, f);
                if (fabs(pred - m->log10tau) < 1e-3)
                    r->flag = 1;
                accept = pred < m->log10tau;
            }
        }
        if (accept)
            pc(w, i, c, x, d2, r);
        else if (w->next[c] == c + 1)
            leaf_pp(w, i, c, r);
        else
            cell_force_mlp(m, c, i, r);
    }
}

void orc_walk_mlp(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                  const int32_t *count, const int32_t *next, const double *M, const double *com,
                  const double *Q, const double *spos, const double *smass, const double *lo,
                  double L, double eps, double theta_lo, double theta_hi, double log10tau,
                  const double *mlp, int64_t nt, const int64_t *targets, double *acc,
                  double *phi, int64_t *npp, int64_t *npc, int32_t *flag)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        mac_ctx m;
        memset(&m, 0, sizeof(m));
        m.w = (walk_ctx){level, begin, count, next, M, com, Q, spos, smass, L, 0.0, eps * eps, 2};
        m.hkey = hkey;
        m.lo = lo;
        m.tlo2 = theta_lo * theta_lo;
        m.thi2 = theta_hi * theta_hi;
        m.eps = eps;
        m.mlp = mlp;
        m.log10tau = log10tau;
        const int64_t i = targets[t];
        walk_acc r;
        memset(&r, 0, sizeof(r));
        if (next[0] == 1)
            leaf_pp(&m.w, i, 0, &r);
        else
            cell_force_mlp(&m, 0, i, &r);
        for (int d = 0; d < 3; ++d)
            acc[3 * t + d] = r.a[d];
        if (phi) phi[t] = r.phi;
        if (npp) npp[t] = r.npp;
        if (npc) npc[t] = r.npc;
        if (flag) flag[t] = r.flag;
    }
}
