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
 * Peano-Hilbert key (Sec. 4.4 names the Peano-Hilbert order as the remedy
 * for the jumps of the Morton order; a method variant).  The index is
 * built one level at a time from the top, following Butz's construction as
 * Hamilton states it (Compact Hilbert Indices, 2006): at every level the
 * point's bits, one per axis (bit j of l is axis j), name the sub-cube it
 * lies in; the current cube's curve is carried onto the standard one by
 * reflecting through its entry corner e and rotating right by d + 1 bits,
 * after which the sub-cubes are visited in Gray-code order, so the
 * sub-cube's rank w is the inverse Gray code of the transformed bits; w is
 * the next n bits of the index; the sub-cube's own curve enters at corner
 * e(w) (the Gray code of the largest even number below w, 0 for w = 0) and
 * leaves along axis g(w) (the trailing set bits of w - 1 for even w, of w
 * for odd w, modulo n), which update e and d.  Axis 0 is x.  In two
 * dimensions this draws Hilbert's own curve; in three, one of the Hilbert
 * curves (the nesting of sub-cubes, the face-adjacency of consecutive
 * cells and the start at the origin are what the tests check).
 * ---------------------------------------------------------------------- */
static unsigned hb_rotr(unsigned x, int r, int n)
{
    r %= n;
    const unsigned mask = (1u << n) - 1u;
    return r == 0 ? x & mask : ((x >> r) | (x << (n - r))) & mask;
}

static unsigned hb_rotl(unsigned x, int r, int n)
{
    r %= n;
    const unsigned mask = (1u << n) - 1u;
    return r == 0 ? x & mask : ((x << r) | (x >> (n - r))) & mask;
}

static unsigned hb_gray(unsigned i) { return i ^ (i >> 1); }

static unsigned hb_gray_inverse(unsigned g)
{
    unsigned i = g;
    for (unsigned s = g >> 1; s; s >>= 1)
        i ^= s;
    return i;
}

static int hb_trailing_ones(unsigned i)
{
    int c = 0;
    while (i & 1u) {
        ++c;
        i >>= 1;
    }
    return c;
}

static unsigned hb_entry(unsigned w) { return w == 0 ? 0u : hb_gray(2u * ((w - 1u) / 2u)); }

static int hb_axis(unsigned w, int n)
{
    if (w == 0)
        return 0;
    return (w & 1u ? hb_trailing_ones(w) : hb_trailing_ones(w - 1u)) % n;
}

uint64_t orc_hilbert(int n, int bits, const uint32_t *q)
{
    unsigned e = 0;
    int d = 0;
    uint64_t h = 0;
    for (int i = bits - 1; i >= 0; --i) {
        unsigned l = 0;
        for (int j = 0; j < n; ++j)
            l |= ((q[j] >> i) & 1u) << j;
        const unsigned w = hb_gray_inverse(hb_rotr(l ^ e, d + 1, n));
        e ^= hb_rotl(hb_entry(w), d + 1, n);
        d = (d + hb_axis(w, n) + 1) % n;
        h = (h << n) | w;
    }
    return h;
}

void orc_keys_hilbert(int64_t n, const double *pos, const double *lo, double L,
                      uint64_t *keys)
{
    const double scale = ldexp(1.0, ORC_LEVELS) / L;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t q[3] = {quantise(pos[3 * i + 0], lo[0], scale),
                               quantise(pos[3 * i + 1], lo[1], scale),
                               quantise(pos[3 * i + 2], lo[2], scale)};
        keys[i] = orc_hilbert(3, ORC_LEVELS, q);
    }
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

static void split_cell(tree_out *t, const uint64_t *keys, const uint64_t *ckeys, int B,
                       int k, uint64_t prefix, int64_t b, int64_t e, int64_t parent)
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
            /* the child's octant: its digit of the Morton cell key */
            const unsigned o = (unsigned)((ckeys[s] >> shift) & 7u);
            if (w)
                t->cmask[id] |= 1 << o;
            split_cell(t, keys, ckeys, B, k + 1, (prefix << 3) | o, s, f, id);
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
    split_cell(&t, sorted_keys, sorted_keys, leaf_size, 0, 0, 0, n, -1);
    return t.m;
}

/* The same tree over bodies sorted by another space-filling curve's keys
 * (the Peano-Hilbert keys): cells are split and ordered by the curve's
 * digits (a curve prefix of k digits names a level-k cube, as a Morton
 * prefix does), and named, as before, by their Morton hashed keys taken
 * from cell_keys (the Morton keys of the same sorted bodies), so that the
 * hashed key, the child mask (by octant) and the cell centre keep their
 * geometric meaning. */
int64_t orc_build_curve(int64_t n, const uint64_t *sorted_keys, const uint64_t *cell_keys,
                        int leaf_size, uint64_t *hkey, int32_t *level, int32_t *begin,
                        int32_t *count, int32_t *next, int32_t *parent, int32_t *cmask)
{
    tree_out t = {0, hkey, level, begin, count, next, parent, cmask};
    split_cell(&t, sorted_keys, cell_keys, leaf_size, 0, 0, 0, n, -1);
    return t.m;
}

/* ------------------------------------------------------------------------
 * Cell moments (Sec. 2.2, truncated multipole expansion): total mass M0,
 * centre of mass (the dipole vanishes about it; the COM is the mass-weighted
 * mean position -- the displayed COM formula omits the division by the
 * mass), and Q_ab = sum m (3 y_a y_b - |y|^2 delta_ab) with y the body's
 * offset from the COM.  Computed per cell directly from its bodies.
 * A massless cell gets its geometric centre as COM and Q = 0.
 * Q layout: xx, xy, xz, yy, yz, zz.  trT (optional): sum m |y|^2, the trace
 * of the second moment about the COM, which the traceless Q does not carry.
 * ---------------------------------------------------------------------- */
void orc_moments(int64_t m, const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                 const int32_t *count, const double *spos, const double *smass,
                 const double *lo, double L, double *M, double *com, double *Q, double *trT)
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
        double q[6] = {0, 0, 0, 0, 0, 0}, tr = 0.0;
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
            tr += mj * r2;
        }
        if (trT)
            trT[c] = tr;
        M[c] = mt;
        com[3 * c + 0] = cx;
        com[3 * c + 1] = cy;
        com[3 * c + 2] = cz;
        for (int a = 0; a < 6; ++a)
            Q[6 * c + a] = q[a];
    }
}

/* ------------------------------------------------------------------------
 * Octopole moments (Sec. 2.2: the next term of the multipole expansion,
 * l = 3), per cell directly from its bodies about its COM:
 *   O_abc = sum m (15 y_a y_b y_c - 3 |y|^2 (y_a d_bc + y_b d_ac + y_c d_ab)),
 * symmetric and traceless (10 components: xxx xxy xxz xyy xyz xzz yyy yyz
 * yzz zzz).  Its potential at x (from the COM) is -O:xxx / (6 r^7), the
 * Legendre term P_3 of 1/|x - y| summed over the bodies.
 * ---------------------------------------------------------------------- */
void orc_octopole(int64_t m, const int32_t *begin, const int32_t *count, const double *spos,
                  const double *smass, const double *com, double *O)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < m; ++c) {
        double o[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t j = begin[c]; j < begin[c] + count[c]; ++j) {
            const double y[3] = {spos[3 * j] - com[3 * c], spos[3 * j + 1] - com[3 * c + 1],
                                 spos[3 * j + 2] - com[3 * c + 2]};
            const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
            static const int ia[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2};
            static const int ib[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2};
            static const int ic[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
            for (int k = 0; k < 10; ++k) {
                const int a = ia[k], b = ib[k], cc = ic[k];
                const double tr = (b == cc ? y[a] : 0.0) + (a == cc ? y[b] : 0.0) +
                                  (a == b ? y[cc] : 0.0);
                o[k] += smass[j] * (15.0 * y[a] * y[b] * y[cc] - 3.0 * r2 * tr);
            }
        }
        for (int k = 0; k < 10; ++k)
            O[10 * c + k] = o[k];
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
 *
 * With the containment guard (a variant, not in the paper) a cell whose
 * closed cube holds the body is opened whatever its opening angle; the flag
 * is also set when the body lies within a relative 1e-6 of a face.  Below
 * theta = 1/sqrt(3) no cell holding the body can pass the test (d is at most
 * the cube's diagonal), so the guard changes nothing there.
 * ---------------------------------------------------------------------- */
typedef struct {
    const int32_t *level, *begin, *count, *next;
    const double *M, *com, *Q;
    const double *spos, *smass;
    double L, theta2, e2;
    int order;
    /* containment guard (opening angle only): hashed keys and the root
     * cube's corner, or guard = 0 */
    const uint64_t *hkey;
    const double *lo;
    int guard;
    /* relative margin of the opening-angle test inside which reduced
     * precision may decide either way (flags the body); 0 means 1e-5 */
    double tol;
    /* order 3: octopole moments per cell (10 each), else NULL */
    const double *O;
} walk_ctx;

static void cell_centre(uint64_t hkey, int k, const double *lo, double L, double c[3]);
static int inside_cell(const double *r, const double *centre, double side);

/* Three-valued reading of one comparison "a < b" taken in reduced
 * precision: +1 surely true, -1 surely false, 0 within a relative tol of
 * the threshold (scale: the magnitude the margin is measured against). */
static int cmp3(double a, double b, double tol, double scale)
{
    if (b - a > tol * scale)
        return 1;
    if (a - b > tol * scale)
        return -1;
    return 0;
}

/* A conjunction of three-valued terms: the decision may flip only if no
 * term is surely false and at least one is uncertain. */
static int and_uncertain(const int *t, int n)
{
    int unc = 0;
    for (int k = 0; k < n; ++k) {
        if (t[k] < 0)
            return 0;
        if (t[k] == 0)
            unc = 1;
    }
    return unc;
}


typedef struct {
    double a[3], phi;
    int64_t npp, npc, ncov;
    int64_t npq; /* particle-cell terms that carry the quadrupole */
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

/* The particle-cell term of cell c for body i up to expansion order `order`
 * (0, 2 or 3). */
static void pc_ord(const walk_ctx *w, int64_t i, int64_t c, const double x[3], double d2,
                   walk_acc *r, int order)
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
    if (order >= 2) {
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
        r->npq += 1;
    }
    if (order >= 3) {
        /* a = (O:xx) / (2 s^7) - 7 (O:xxx) x / (6 s^9), the gradient of
         * O:xxx / (6 s^7) */
        const double *o = &w->O[10 * c];
        const double xx = x[0] * x[0], yy = x[1] * x[1], zz = x[2] * x[2];
        const double xy = x[0] * x[1], xz = x[0] * x[2], yz = x[1] * x[2];
        const double vx = o[0] * xx + o[3] * yy + o[5] * zz + 2.0 * (o[1] * xy + o[2] * xz + o[4] * yz);
        const double vy = o[1] * xx + o[6] * yy + o[8] * zz + 2.0 * (o[3] * xy + o[4] * xz + o[7] * yz);
        const double vz = o[2] * xx + o[7] * yy + o[9] * zz + 2.0 * (o[4] * xy + o[5] * xz + o[8] * yz);
        const double t3 = x[0] * vx + x[1] * vy + x[2] * vz;
        const double inv7 = inv3 * inv2 * inv2;
        const double inv9 = inv7 * inv2;
        r->a[0] += 0.5 * vx * inv7 - (7.0 / 6.0) * t3 * x[0] * inv9;
        r->a[1] += 0.5 * vy * inv7 - (7.0 / 6.0) * t3 * x[1] * inv9;
        r->a[2] += 0.5 * vz * inv7 - (7.0 / 6.0) * t3 * x[2] * inv9;
        r->phi -= t3 * inv7 / 6.0;
    }
    (void)i;
    r->npc += 1;
    r->ncov += w->count[c];
}

static void pc(const walk_ctx *w, int64_t i, int64_t c, const double x[3], double d2, walk_acc *r)
{
    pc_ord(w, i, c, x, d2, r, w->order);
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
        int terms[2] = {cmp3(lhs, rhs, w->tol > 0.0 ? w->tol : 1e-5, lhs), 1};
        int in = 0;
        if (w->guard) { /* a cell that holds the body is opened */
            double centre[3];
            cell_centre(w->hkey[c], w->level[c], w->lo, w->L, centre);
            terms[1] = -1;
            for (int a = 0; a < 3; ++a) {
                const int o3 = cmp3(0.5 * side, fabs(w->spos[3 * i + a] - centre[a]), 1e-6, side);
                if (o3 > terms[1])
                    terms[1] = o3;
            }
            in = inside_cell(&w->spos[3 * i], centre, side);
        }
        if (and_uncertain(terms, 2))
            r->flag = 1;
        if (lhs < rhs && !in)
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
              int64_t *npp, int64_t *npc, int64_t *ncov, int32_t *flag, const uint64_t *hkey,
              const double *lo, int guard, double tol, const double *O)
{
    walk_ctx w = {level, begin, count, next, M, com, Q, spos, smass,
                  L, theta * theta, eps * eps, order, hkey, lo, guard, tol, O};
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
 * Network helpers and the error budget.
 *
 * The error budget accepts a multi-body cell for body i iff
 * l^2 < theta_max^2 d^2, the body lies outside the cell, and
 * M l^3 < tau |a_i| d^5 (the quadrupole term's error taken as
 * (l/d)^3 M/d^2, the next order of the expansion of Sec. 2.2).  The
 * network helpers evaluate the learned criterion's network with bf16 or
 * fp16 operands as the MFMA inference does (see the learned section below).
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

/* SplitMix64 (Steele, Lea & Flood 2014): the finaliser applied to x. */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* keep a candidate (hash key i, node c) with probability p */
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

/* round an FP32 value to IEEE binary16, nearest even: 11 significant bits
 * for normal values (|x| >= 2^-14), a fixed spacing of 2^-24 below, and
 * infinity from 65520 (the midpoint between 65504 and 2^16) up */
static double f16r(double x)
{
    const float f = (float)x;
    const double a = fabs((double)f);
    if (a == 0.0 || a != a)
        return (double)f;
    if (a >= 65520.0)
        return copysign(INFINITY, (double)f);
    int e;
    frexp(a, &e); /* a = m 2^e, m in [0.5, 1) */
    int q = e - 11;
    if (q < -24)
        q = -24;
    const double s = ldexp(1.0, q);
    return copysign(nearbyint(a / s) * s, (double)f);
}

/* The network as the MFMA inference evaluates it (see oracle/mlp.py), with
 * rounding rnd of the operands (bf16 or fp16): parameters W1[32][10] b1[32]
 * W2[32][32] b2[32] w3[32] b3. */
static double mlp_rounded(const double *p, const double *f, double (*rnd)(double))
{
    const double *W1 = p, *b1 = p + 320, *W2 = p + 352, *b2 = p + 1376, *w3 = p + 1408;
    const double b3 = (double)(float)p[1440];
    double h1[32], out = 0.0;
    for (int u = 0; u < 32; ++u) {
        double s = rnd(b1[u]);
        for (int k = 0; k < 10; ++k)
            s += rnd(W1[u * 10 + k]) * rnd(f[k]);
        h1[u] = rnd(s > 0.0 ? s : 0.0);
    }
    for (int u = 0; u < 32; ++u) {
        double s = (double)(float)b2[u];
        for (int k = 0; k < 32; ++k)
            s += rnd(W2[u * 32 + k]) * h1[k];
        if (s > 0.0)
            out += (double)(float)w3[u] * s;
    }
    return out + b3;
}

double orc_mlp_bf16(const double *p, const double *f) { return mlp_rounded(p, f, bf16r); }
double orc_mlp_f16(const double *p, const double *f) { return mlp_rounded(p, f, f16r); }
double orc_f16r(double x) { return f16r(x); }

typedef struct {
    walk_ctx w;
    const uint64_t *hkey;
    const double *lo;
    double tmax2;
    const double *kc;  /* per cell M l^3 */
    double tau, anorm; /* tau and |a_i| of the current body */
} mac_ctx;

/* The quadrupole term a particle-cell term drops when it keeps the monopole
 * only (order 0): a_Q = Q x / s^5 - (5/2) (x.Q.x) x / s^7 (Sec. 2.2, R10).
 * With |Q y| <= |Q|_2 |y| <= |Q|_F |y| and |x| <= s,
 *   |a_Q| <= |Q|_F |x| / s^5 + (5/2) |Q|_F |x|^3 / s^7 <= (7/2) |Q|_F / s^4.
 * The error budget with monopole terms charges a cell this bound at the
 * (group) distance d plus the next order's estimate M l^3 / d^5:
 *   M l^3 + (7/2) |Q|_F d < tau a d^5. */
#define ORC_QUAD_BOUND 3.5
static double q_frobenius(const double *q)
{
    return sqrt(q[0] * q[0] + q[3] * q[3] + q[5] * q[5] +
                2.0 * (q[1] * q[1] + q[2] * q[2] + q[4] * q[4]));
}

/* Mixed order (order 1 in the budget walks): a cell accepted with its
 * monopole where the budget charged with the dropped quadrupole's bound
 * holds, else with the quadrupole where the plain budget holds, else
 * opened.  Both kinds of term meet the same budget; the quadrupole costs
 * more arithmetic than the monopole and less than opening the cell. */
#define ORC_ORDER_MIXED 1

/* The budget decision for one cell: 0 open, else the order of the term
 * (0 or 2) it is accepted with.  geo: the geometric terms (angle, outside)
 * as three-valued tests, n_geo of them, and their conjunction ok; kc the
 * cell's M l^3, qb its (7/2) |Q|_F, d the distance, rhs tau a d^5.  Sets
 * *unc if a near-threshold test could change the decision or the order. */
static int budget_choice(int order, const int *geo, int n_geo, int ok, double kc, double qb,
                         double d, double rhs, double tol, int *unc)
{
    int t[4];
    for (int k = 0; k < n_geo; ++k)
        t[k] = geo[k];
    const double lhs_m = kc + qb * d; /* monopole: the quadrupole's bound charged */
    const int mono = order == 0 || order == ORC_ORDER_MIXED; /* monopole terms allowed */
    const int high = order != 0; /* terms with the quadrupole (and above) allowed */
    if (high) {
        t[n_geo] = cmp3(kc, rhs, tol, kc);
        if (and_uncertain(t, n_geo + 1))
            *unc = 1;
    }
    if (mono) {
        t[n_geo] = cmp3(lhs_m, rhs, tol, lhs_m);
        if (and_uncertain(t, n_geo + 1))
            *unc = 1;
    }
    if (!ok)
        return -1;
    if (mono && lhs_m < rhs)
        return 0;
    if (high && kc < rhs)
        return order == ORC_ORDER_MIXED ? 2 : order;
    return -1;
}

/* Per cell: M l^3, the error budget's k_C M l^3 with k_C = 1. */
void orc_cell_kc(int64_t m, const int32_t *level, const double *M, double L, double *kc)
{
    for (int64_t c = 0; c < m; ++c) {
        const double side = ldexp(L, -level[c]);
        kc[c] = M[c] * side * side * side;
    }
}

/* Tree walk with the learned criterion: a multi-body cell is accepted iff
 * l^2 < theta_max^2 d^2, the body is outside the cell, and
 * kc_C < tau |a_i| d^5 (one-body cells and rejected leaves
 * particle-particle, rejected internal cells opened).  The flag marks tests
 * within a relative 1e-5 of a threshold and bodies within 1e-6 l of a face
 * of a cell they are tested against. */
static void cell_force_kc(mac_ctx *m, int64_t node, int64_t i, walk_acc *r)
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
        const double rhs = m->tau * m->anorm * d2 * d2 * sqrt(d2);
        double centre[3];
        cell_centre(m->hkey[c], w->level[c], m->lo, w->L, centre);
        int out = -1; /* three-valued "the body lies outside the cube" */
        for (int a = 0; a < 3; ++a) {
            const int o3 = cmp3(0.5 * side, fabs(w->spos[3 * i + a] - centre[a]), 1e-6, side);
            if (o3 > out)
                out = o3;
        }
        const int geo[2] = {cmp3(s2, m->tmax2 * d2, 1e-5, s2), out};
        const int in = inside_cell(&w->spos[3 * i], centre, side);
        /* monopole terms (order 0, or mixed): the dropped quadrupole's
         * bound charged as well */
        const int ord = budget_choice(w->order, geo, 2, s2 < m->tmax2 * d2 && !in, m->kc[c],
                                      ORC_QUAD_BOUND * q_frobenius(&w->Q[6 * c]), sqrt(d2), rhs,
                                      1e-5, &r->flag);
        if (ord >= 0)
            pc_ord(w, i, c, x, d2, r, ord);
        else if (w->next[c] == c + 1)
            leaf_pp(w, i, c, r);
        else
            cell_force_kc(m, c, i, r);
    }
}

void orc_walk_kc(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                 const int32_t *count, const int32_t *next, const double *M, const double *com,
                 const double *Q, const double *spos, const double *smass, const double *lo,
                 double L, double eps, double theta_max,
                 double tau, const double *kc, const double *anorm, int64_t nt,
                 const int64_t *targets, double *acc, double *phi, int64_t *npp, int64_t *npc,
                 int64_t *ncov, int32_t *flag, int order, int64_t *npq)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        mac_ctx m;
        memset(&m, 0, sizeof(m));
        m.w = (walk_ctx){level, begin, count, next, M, com, Q, spos, smass, L, 0.0, eps * eps,
                         order};
        m.hkey = hkey;
        m.lo = lo;
        m.tmax2 = theta_max * theta_max;
        m.kc = kc;
        m.tau = tau;
        const int64_t i = targets[t];
        m.anorm = anorm[i];
        walk_acc r;
        memset(&r, 0, sizeof(r));
        if (next[0] == 1)
            leaf_pp(&m.w, i, 0, &r);
        else
            cell_force_kc(&m, 0, i, &r);
        for (int d = 0; d < 3; ++d)
            acc[3 * t + d] = r.a[d];
        if (phi) phi[t] = r.phi;
        if (npp) npp[t] = r.npp;
        if (npc) npc[t] = r.npc;
        if (npq) npq[t] = r.npq;
        if (ncov) ncov[t] = r.ncov;
        if (flag) flag[t] = r.flag;
    }
}

/* ========================================================================
 * Group walk: one acceptance decision per cell for a whole group of bodies.
 *
 * The bodies of sorted ranks [t0, t1) are split into consecutive groups of
 * G.  A group's box is the axis-aligned bounding box of its bodies (centre
 * bc, half extent bh).  For a multi-body cell C with side l, centre c and
 * centre of mass x_C, the group distance is the distance from x_C to the
 * box, d_g^2 = sum_a max(0, |x_C,a - bc_a| - bh_a)^2, and C overlaps the
 * group when its closed cube meets the box (|c_a - bc_a| <= l/2 + bh_a on
 * every axis).  C is accepted for every body of the group iff it does not
 * overlap and
 *   mode 0 (opening angle):  l^2 < theta^2 d_g^2;
 *   mode 1 (error budget):   l^2 < theta_max^2 d_g^2 and
 *                            kc_C < tau a_min d_g^5,  a_min = min |a_i|
 *                            over the group.
 * Accepted cells give every body of the group a particle-cell term with its
 * own distance; one-body cells and rejected leaves particle-particle terms
 * (a body skips itself); rejected internal cells are opened; the root is
 * always opened.  Since d_g <= d for every body of the group, the group
 * accepts a cell only where each of its bodies would.  With G = 1 the box
 * is the body itself: d_g = d, the overlap test is "the body lies in the
 * closed cube", and mode 0 is the per-body walk of Sec. 3 for theta below
 * 1/sqrt(3) (where no accepted cell can contain the body).
 *
 * The work of a group is the number of particle-cell terms plus the number
 * of bodies of its particle-particle cells (its own bodies included), the
 * same for each body of the group.  A group whose work exceeds cap is
 * walked per body instead, with the same criterion: the walk of Sec. 3 at
 * theta (mode 0), or the per-body error-budget walk (mode 1).
 *
 * With split set, a group that straddles a jump of the space-filling curve
 * is first cut into runs of consecutive bodies, each walked as a group of
 * its own (box, decisions, cap).  From the left: the run is [lo, g1); while
 * it holds two or more bodies and its common cell (level = the smallest
 * common-prefix length, in octal digits, of adjacent keys inside it) lies
 * more than two levels above its shallowest leaf, it is cut before its
 * first adjacent pair with that smallest common prefix.  The run found is
 * walked and the next starts where it ended.
 *
 * flag[t] is set for every body of a group that met a test within a
 * relative tol of a threshold, or a cube face within tol * l of the box.
 * ====================================================================== */
typedef struct {
    walk_ctx w;
    const uint64_t *hkey;
    const double *lo, *kc;
    int mode;
    double th2, tmax2, tau, amin, tol;
    double bc[3], bh[3];
    int64_t g0, g1;
    walk_acc *r; /* one per body of the group */
    int flag;
    int64_t work;
    /* mode 2 (learned): network parameters (fp16 operands if f16, else
     * bf16), softening, log10(tau amin) */
    const double *params;
    int f16;
    double eps, lt;
} group_ctx;

static int learned_term(const group_ctx *g, int64_t c, double side, double dg2, int *accept);

static void group_cell(group_ctx *g, int64_t node)
{
    const walk_ctx *w = &g->w;
    for (int64_t c = node + 1; c < w->next[node]; c = w->next[c]) {
        if (w->count[c] == 1) {
            for (int64_t i = g->g0; i < g->g1; ++i)
                if (w->begin[c] != i)
                    pp(w, i, w->begin[c], &g->r[i - g->g0]);
            g->work += 1;
            continue;
        }
        const double side = ldexp(w->L, -w->level[c]);
        double centre[3], dg2 = 0.0;
        int overlap = 1, sep = -1; /* sep: three-valued "cube misses the box" */
        cell_centre(g->hkey[c], w->level[c], g->lo, w->L, centre);
        for (int a = 0; a < 3; ++a) {
            const double gap = fabs(centre[a] - g->bc[a]) - (0.5 * side + g->bh[a]);
            if (gap > 0.0)
                overlap = 0;
            const int s3 = cmp3(0.0, gap, g->tol, side);
            if (s3 > sep)
                sep = s3;
            const double t = fabs(w->com[3 * c + a] - g->bc[a]) - g->bh[a];
            if (t > 0.0)
                dg2 += t * t;
        }
        const double s2 = side * side;
        const double lim2 = (g->mode == 0 ? g->th2 : g->tmax2) * dg2;
        int accept = !overlap && s2 < lim2;
        int terms[3] = {sep, cmp3(s2, lim2, g->tol, s2), 1};
        int ord = w->order;
        if (g->mode == 1) {
            /* monopole terms (order 0, or mixed): the dropped quadrupole's
             * bound charged as well */
            const double rhs = g->tau * g->amin * dg2 * dg2 * sqrt(dg2);
            ord = budget_choice(w->order, terms, 2, accept, g->kc[c],
                                ORC_QUAD_BOUND * q_frobenius(&w->Q[6 * c]), sqrt(dg2), rhs,
                                g->tol, &g->flag);
            accept = ord >= 0;
        } else if (g->mode == 2 && sep >= 0 && terms[1] >= 0) {
            int acc_l = 0;
            terms[2] = learned_term(g, c, side, dg2, &acc_l);
            accept = accept && acc_l;
        }
        if (g->mode != 1 && and_uncertain(terms, 3))
            g->flag = 1;
        if (accept) {
            for (int64_t i = g->g0; i < g->g1; ++i) {
                double x[3];
                for (int d = 0; d < 3; ++d)
                    x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
                pc_ord(w, i, c, x, x[0] * x[0] + x[1] * x[1] + x[2] * x[2], &g->r[i - g->g0],
                       ord);
            }
            g->work += 1;
        } else if (w->next[c] == c + 1) {
            for (int64_t i = g->g0; i < g->g1; ++i)
                leaf_pp(w, i, c, &g->r[i - g->g0]);
            g->work += w->count[c];
        } else {
            group_cell(g, c);
        }
    }
}

/* Outputs indexed by t - t0 for t in [t0, t1). */
static void walk_one_group(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                           const int32_t *count, const int32_t *next, const double *M,
                           const double *com, const double *Q, const double *spos,
                           const double *smass, const double *lo, double L, double eps,
                           int order, int mode, double theta, double theta_max, double tau,
                           const double *kc, const double *anorm, const double *params,
                           int f16, int64_t r0, int64_t r1, int64_t t0, int64_t cap, double tol,
                           double *acc, double *phi, int64_t *npp, int64_t *npc, int64_t *ncov,
                           int32_t *flag, const double *O, int64_t *npq);

static void group_run(group_ctx *g, int64_t r0, int64_t r1, const double *anorm, walk_acc *r);

/* common octal digits of two keys (21 if equal) */
static int key_lcp(uint64_t a, uint64_t b)
{
    const uint64_t x = a ^ b;
    if (!x)
        return ORC_LEVELS;
    int lz = 0;
    while (!((x << lz) & ((uint64_t)1 << 63)))
        ++lz;
    return (lz - 1) / 3;
}

void orc_walk_group(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                    const int32_t *count, const int32_t *next, const double *M,
                    const double *com, const double *Q, const double *spos, const double *smass,
                    const double *lo, double L, double eps, int order, int mode, double theta,
                    double theta_max, double tau, const double *kc, const double *anorm,
                    const double *params, int f16, int64_t G, int64_t t0, int64_t t1,
                    int64_t cap, double tol,
                    const uint64_t *skeys, const int32_t *leaf_level, int split, double *acc,
                    double *phi, int64_t *npp, int64_t *npc, int64_t *ncov, int32_t *flag,
                    const double *O, int64_t *npq)
{
    const int64_t ng = (t1 - t0 + G - 1) / G;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t gi = 0; gi < ng; ++gi) {
        const int64_t g0 = t0 + gi * G, g1 = g0 + G < t1 ? g0 + G : t1;
        int64_t a = g0;
        while (a < g1) {
            int64_t b = g1;
            while (split && b - a >= 2) {
                int kanc = 127, kleaf = 127;
                int64_t cut = -1;
                for (int64_t j = a + 1; j < b; ++j) {
                    const int d = key_lcp(skeys[j - 1], skeys[j]);
                    if (d < kanc) {
                        kanc = d;
                        cut = j;
                    }
                }
                for (int64_t j = a; j < b; ++j)
                    if (leaf_level[j] < kleaf)
                        kleaf = leaf_level[j];
                if (kanc >= kleaf - 2)
                    break;
                b = cut;
            }
            walk_one_group(level, hkey, begin, count, next, M, com, Q, spos, smass, lo, L, eps,
                           order, mode, theta, theta_max, tau, kc, anorm, params, f16, a, b, t0,
                           cap, tol, acc, phi, npp, npc, ncov, flag, O, npq);
            a = b;
        }
    }
}

/* One group (or run): the bodies of sorted rank [r0, r1), outputs at rank - t0. */
static void walk_one_group(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                           const int32_t *count, const int32_t *next, const double *M,
                           const double *com, const double *Q, const double *spos,
                           const double *smass, const double *lo, double L, double eps,
                           int order, int mode, double theta, double theta_max, double tau,
                           const double *kc, const double *anorm, const double *params,
                           int f16, int64_t r0, int64_t r1, int64_t t0, int64_t cap, double tol,
                           double *acc, double *phi, int64_t *npp, int64_t *npc, int64_t *ncov,
                           int32_t *flag, const double *O, int64_t *npq)
{
    {
        group_ctx g;
        memset(&g, 0, sizeof(g));
        g.w = (walk_ctx){level, begin, count, next, M, com, Q, spos, smass, L, 0.0, eps * eps,
                         order};
        g.w.O = O;
        g.hkey = hkey;
        g.lo = lo;
        g.kc = kc;
        g.mode = mode;
        g.th2 = theta * theta;
        g.tmax2 = theta_max * theta_max;
        g.tau = tau;
        g.tol = tol;
        g.params = params;
        g.f16 = f16;
        g.eps = eps;
        g.r = calloc((size_t)(r1 - r0), sizeof(walk_acc));
        group_run(&g, r0, r1, anorm, g.r);
        /* with no uncertain group decision the work is exact, and so is the
         * choice to walk per body: then each body's flag is its own */
        const int gflag = g.flag;
        const int per_body = g.work > cap;
        if (per_body) { /* too spread out for one decision: per body */
            memset(g.r, 0, (size_t)(r1 - r0) * sizeof(walk_acc));
            for (int64_t i = r0; i < r1; ++i) {
                walk_acc *r = &g.r[i - r0];
                if (mode == 2) { /* the learned decision with the body as the group */
                    group_ctx g1 = g;
                    group_run(&g1, i, i + 1, anorm, r);
                    r->flag = g1.flag;
                    continue;
                }
                if (mode == 0) {
                    walk_ctx w1 = g.w;
                    w1.theta2 = theta * theta;
                    w1.tol = tol;
                    if (next[0] == 1)
                        leaf_pp(&w1, i, 0, r);
                    else
                        cell_force(&w1, 0, i, r);
                } else {
                    mac_ctx mc;
                    memset(&mc, 0, sizeof(mc));
                    mc.w = g.w;
                    mc.hkey = hkey;
                    mc.lo = lo;
                    mc.tmax2 = theta_max * theta_max;
                    mc.kc = kc;
                    mc.tau = tau;
                    mc.anorm = anorm[i];
                    if (next[0] == 1)
                        leaf_pp(&mc.w, i, 0, r);
                    else
                        cell_force_kc(&mc, 0, i, r);
                }
            }
        }
        for (int64_t i = g.g0; i < g.g1; ++i) {
            const walk_acc *r = &g.r[i - g.g0];
            const int64_t o = i - t0;
            for (int d = 0; d < 3; ++d)
                acc[3 * o + d] = r->a[d];
            if (phi) phi[o] = r->phi;
            if (npp) npp[o] = r->npp;
            if (npc) npc[o] = r->npc;
            if (npq) npq[o] = r->npq;
            if (ncov) ncov[o] = r->ncov;
            if (flag) flag[o] = gflag || (per_body && r->flag);
        }
        free(g.r);
    }
}

/* Walks the bodies of sorted rank [r0, r1) as one group: box, smallest
 * norm, decisions; accumulators r[0 .. r1 - r0), work and flag in g. */
static void group_run(group_ctx *g, int64_t r0, int64_t r1, const double *anorm, walk_acc *r)
{
    const walk_ctx *w = &g->w;
    g->g0 = r0;
    g->g1 = r1;
    g->r = r;
    g->work = 0;
    g->flag = 0;
    double bl[3] = {INFINITY, INFINITY, INFINITY}, bu[3] = {-INFINITY, -INFINITY, -INFINITY};
    g->amin = INFINITY;
    for (int64_t i = r0; i < r1; ++i) {
        for (int a = 0; a < 3; ++a) {
            bl[a] = fmin(bl[a], w->spos[3 * i + a]);
            bu[a] = fmax(bu[a], w->spos[3 * i + a]);
        }
        if (anorm)
            g->amin = fmin(g->amin, anorm[i]);
    }
    for (int a = 0; a < 3; ++a) {
        g->bc[a] = 0.5 * (bl[a] + bu[a]);
        g->bh[a] = 0.5 * (bu[a] - bl[a]);
    }
    g->lt = anorm ? log10(g->tau * g->amin) : 0.0;
    if (w->next[0] == 1) {
        for (int64_t i = r0; i < r1; ++i)
            leaf_pp(w, i, 0, &r[i - r0]);
        g->work = w->count[0];
    } else {
        group_cell(g, 0);
    }
}

/* ========================================================================
 * Learned acceptance criterion, one decision per (group, cell).
 *
 * A network predicts the error a cell's particle-cell term (order 2) makes
 * on a group of bodies: the largest |a_pc,i - a_exact,i| over the group in
 * units of the error budget's model M l^3 / d_g^5 (the next order of the
 * expansion at the group's box), as log10 -- a coefficient k_C per (group,
 * cell).  The cell is accepted for the group iff its cube misses the box,
 * l^2 < theta_max^2 d_g^2, and
 *     pred + log10(M l^3 / d_g^5) < log10(tau a_min),
 * i.e. iff the predicted error is below tau times the group's smallest
 * |a_i|: the error budget with k_C = 10^pred.  A group of one body is the
 * per-body criterion.
 *
 * Features of (box, cell), all scale-free (l side, d_g distance from the
 * COM to the box, d_c to the box centre, h the box's half-diagonal,
 * n the unit vector from the box centre to the COM, g = COM - cell centre,
 * Q the traceless quadrupole, n_C the body count):
 *   f0 log2(l/d_g) in [-8, 8]       f1 min(log2(d_c/d_g), 8)
 *   f2 h / (h + d_g)                f3 n.Q.n / (M l^2)
 *   f4 |Q|_F / (M l^2)              f5 g.n / l
 *   f6 |g| / l                      f7 log2(n_C) / 21
 *   f8 min(eps / d_g, 1)            f9 1 for a leaf, else 0
 * ====================================================================== */

void orc_gfeatures(const double *bl, const double *bu, const double *centre, double side,
                   const double *com, double M, const double *Q, int count, int is_leaf,
                   double eps, double *f)
{
    double u[3], g[3], dc2 = 0.0, dg2 = 0.0, h2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double bc = 0.5 * (bl[a] + bu[a]), bh = 0.5 * (bu[a] - bl[a]);
        u[a] = com[a] - bc;
        dc2 += u[a] * u[a];
        const double t = fabs(u[a]) - bh;
        if (t > 0.0)
            dg2 += t * t;
        h2 += bh * bh;
        g[a] = com[a] - centre[a];
    }
    const double dc = sqrt(dc2), dg = sqrt(dg2), h = sqrt(h2);
    double n[3] = {0.0, 0.0, 0.0};
    if (dc > 0.0)
        for (int a = 0; a < 3; ++a)
            n[a] = u[a] / dc;
    const double ml2 = M * side * side;
    const double q[3][3] = {{Q[0], Q[1], Q[2]}, {Q[1], Q[3], Q[4]}, {Q[2], Q[4], Q[5]}};
    double nqn = 0.0, qf = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            nqn += n[a] * q[a][b] * n[b];
            qf += q[a][b] * q[a][b];
        }
    double f0 = dg > 0.0 ? log2(side / dg) : 8.0;
    f[0] = f0 < -8.0 ? -8.0 : (f0 > 8.0 ? 8.0 : f0);
    const double f1 = dg > 0.0 ? log2(dc / dg) : 8.0;
    f[1] = f1 > 8.0 ? 8.0 : f1;
    f[2] = h + dg > 0.0 ? h / (h + dg) : 0.0;
    f[3] = ml2 > 0.0 ? nqn / ml2 : 0.0;
    f[4] = ml2 > 0.0 ? sqrt(qf) / ml2 : 0.0;
    f[5] = (g[0] * n[0] + g[1] * n[1] + g[2] * n[2]) / side;
    f[6] = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) / side;
    f[7] = log2((double)count) / 21.0;
    f[8] = dg > 0.0 ? (eps / dg < 1.0 ? eps / dg : 1.0) : 1.0;
    f[9] = is_leaf ? 1.0 : 0.0;
}

/* The network as the MFMA inference evaluates it (bf16 or fp16 operands of
 * both hidden layers by rnd, sums in FP32 there, FP64 here) from given
 * rounded features fr; h1 receives the rounded hidden layer, z1 its sums. */
static double gnet_fwd(const double *p, const double *fr, double (*rnd)(double), double *h1,
                       double *z1, double *z2)
{
    const double *W1 = p, *b1 = p + 320, *W2 = p + 352, *b2 = p + 1376, *w3 = p + 1408;
    double out = (double)(float)p[1440];
    for (int j = 0; j < 32; ++j) {
        double s = rnd(b1[j]);
        for (int k = 0; k < 10; ++k)
            s += rnd(W1[j * 10 + k]) * fr[k];
        z1[j] = s;
        h1[j] = rnd(s > 0.0 ? s : 0.0);
    }
    for (int u = 0; u < 32; ++u) {
        double s = (double)(float)b2[u];
        for (int j = 0; j < 32; ++j)
            s += rnd(W2[u * 32 + j]) * h1[j];
        z2[u] = s;
        if (s > 0.0)
            out += (double)(float)w3[u] * s;
    }
    return out;
}

/* The network's output from the features f, and *delta, a bound on how far
 * an evaluation of the same features in FP32 (features computed in FP32,
 * sums in FP32) may move it:
 *  - a feature computed in FP32 lies within 4e-6 (|f| + 1) of the exact
 *    one; if that interval holds a rounding midpoint, the operand may round
 *    to the other neighbour: the output with that operand is evaluated and
 *    the difference added;
 *  - a hidden unit's FP32 sum lies within (terms + 1) 2^-24 times the sum
 *    of its absolute terms of the exact one; if that interval holds a
 *    rounding midpoint (or 0), the same;
 *  - the second layer's and the output's FP32 sums move the output by at
 *    most their error bound times |w3| (ReLU is 1-Lipschitz).
 * Flips are taken one at a time (first order; two flips in one evaluation
 * are rarer still). */
static double gnet_bound(const double *p, const double *f, double *delta, double (*rnd)(double))
{
    const double *W1 = p, *b1 = p + 320, *W2 = p + 352, *w3 = p + 1408;
    const double u24 = ldexp(1.0, -24);
    double fr[10], h1[32], z1[32], z2[32], h1x[32], z1x[32], z2x[32];
    for (int k = 0; k < 10; ++k)
        fr[k] = rnd(f[k]);
    const double out = gnet_fwd(p, fr, rnd, h1, z1, z2);
    double d = 0.0;
    for (int k = 0; k < 10; ++k) {
        const double m = 4e-6 * (fabs(f[k]) + 1.0);
        const double lo = rnd(f[k] - m), hi = rnd(f[k] + m);
        if (lo == hi)
            continue;
        double alt[10];
        memcpy(alt, fr, sizeof(alt));
        alt[k] = fr[k] == lo ? hi : lo;
        d += fabs(gnet_fwd(p, alt, rnd, h1x, z1x, z2x) - out);
    }
    for (int j = 0; j < 32; ++j) {
        double a = fabs(rnd(b1[j]));
        for (int k = 0; k < 10; ++k)
            a += fabs(rnd(W1[j * 10 + k]) * fr[k]);
        const double e = 12.0 * u24 * a;
        const double lo = rnd(z1[j] - e > 0.0 ? z1[j] - e : 0.0);
        const double hi = rnd(z1[j] + e > 0.0 ? z1[j] + e : 0.0);
        if (lo == hi)
            continue;
        /* the output with unit j at its other rounding */
        const double hj = h1[j] == lo ? hi : lo;
        double alt = (double)(float)p[1440];
        for (int u = 0; u < 32; ++u) {
            const double s = z2[u] + rnd(W2[u * 32 + j]) * (hj - h1[j]);
            if (s > 0.0)
                alt += (double)(float)w3[u] * s;
        }
        d += fabs(alt - out);
    }
    double sum_out = fabs((double)(float)p[1440]);
    for (int u = 0; u < 32; ++u) {
        double a = fabs((double)(float)p[1376 + u]);
        for (int j = 0; j < 32; ++j)
            a += fabs(rnd(W2[u * 32 + j]) * h1[j]);
        d += fabs((double)(float)w3[u]) * 34.0 * u24 * a;
        if (z2[u] > 0.0)
            sum_out += fabs((double)(float)w3[u] * z2[u]);
    }
    d += 34.0 * u24 * sum_out;
    *delta = d;
    return out;
}

double orc_gnet_bound(const double *p, const double *f, double *delta, int f16)
{
    return gnet_bound(p, f, delta, f16 ? f16r : bf16r);
}

/* Three-valued learned term of cell c for group g (1 surely accepted, -1
 * surely rejected, 0 uncertain), the decision taken here in *accept. */
static int learned_term(const group_ctx *g, int64_t c, double side, double dg2, int *accept)
{
    const walk_ctx *w = &g->w;
    *accept = 0;
    if (!(dg2 > 0.0) || !(w->M[c] > 0.0))
        return -1;
    double centre[3], bl[3], bu[3], f[10], delta;
    cell_centre(g->hkey[c], w->level[c], g->lo, w->L, centre);
    for (int a = 0; a < 3; ++a) {
        bl[a] = g->bc[a] - g->bh[a];
        bu[a] = g->bc[a] + g->bh[a];
    }
    orc_gfeatures(bl, bu, centre, side, &w->com[3 * c], w->M[c], &w->Q[6 * c], w->count[c],
                  w->next[c] == c + 1, g->eps, f);
    const double pred = gnet_bound(g->params, f, &delta, g->f16 ? f16r : bf16r);
    const double lm = log10(w->M[c]), ls = 1.5 * log10(side * side), ld = 2.5 * log10(dg2);
    const double lhs = pred + lm + ls - ld;
    *accept = lhs < g->lt;
    const double margin =
        delta + g->tol * (fabs(pred) + fabs(lm) + fabs(ls) + fabs(ld) + fabs(g->lt) + 1.0);
    if (g->lt - lhs > margin)
        return 1;
    if (lhs - g->lt > margin)
        return -1;
    return 0;
}

/* ---- training pairs of the learned criterion */

/* label of cell c for the bodies [g0, g1): log10 of the largest
 * |a_pc,i - a_exact,i| d_g^5 / (M l^3), floored at 1e-12 */
static double group_label(const walk_ctx *w, int64_t c, int64_t g0, int64_t g1, double dg2)
{
    const double side = ldexp(w->L, -w->level[c]);
    double emax = 0.0;
    for (int64_t i = g0; i < g1; ++i) {
        walk_acc ex, ap;
        memset(&ex, 0, sizeof(ex));
        memset(&ap, 0, sizeof(ap));
        leaf_pp(w, i, c, &ex);
        double x[3];
        for (int d = 0; d < 3; ++d)
            x[d] = w->spos[3 * i + d] - w->com[3 * c + d];
        pc(w, i, c, x, x[0] * x[0] + x[1] * x[1] + x[2] * x[2], &ap);
        double e = 0.0;
        for (int d = 0; d < 3; ++d)
            e += (ap.a[d] - ex.a[d]) * (ap.a[d] - ex.a[d]);
        if (e > emax)
            emax = e;
    }
    double v = sqrt(emax) * dg2 * dg2 * sqrt(dg2) / (w->M[c] * side * side * side);
    if (!(v > 1e-12))
        v = 1e-12;
    return log10(v);
}

typedef struct {
    walk_ctx w;
    const uint64_t *hkey;
    const double *lo;
    double tlo2, tmax2, eps, keep;
    uint64_t seed;
    int64_t g0, g1, cap, slot0, k;
    double bl[3], bu[3], bc[3], bh[3];
    double *feat, *label;
    int32_t *node;
} gsample_ctx;

/* Candidates of a group: a walk that leaves cells with l < theta_lo d_g
 * alone and opens every other cell; each multi-body cell whose cube misses
 * the box with theta_lo d_g <= l < theta_max d_g is a candidate, kept by
 * the hash of (seed, first rank of the group, node) with probability keep. */
static void gsample_walk(gsample_ctx *m, int64_t node)
{
    const walk_ctx *w = &m->w;
    for (int64_t c = node + 1; c < w->next[node]; c = w->next[c]) {
        if (w->count[c] == 1)
            continue;
        const double side = ldexp(w->L, -w->level[c]);
        double centre[3], dg2 = 0.0;
        int overlap = 1;
        cell_centre(m->hkey[c], w->level[c], m->lo, w->L, centre);
        for (int a = 0; a < 3; ++a) {
            if (fabs(centre[a] - m->bc[a]) - (0.5 * side + m->bh[a]) > 0.0)
                overlap = 0;
            const double t = fabs(w->com[3 * c + a] - m->bc[a]) - m->bh[a];
            if (t > 0.0)
                dg2 += t * t;
        }
        const double s2 = side * side;
        if (!overlap && s2 < m->tlo2 * dg2)
            continue;
        if (!overlap && s2 < m->tmax2 * dg2 && w->M[c] > 0.0 &&
            keep_pair(m->seed, m->g0, c, m->keep) && m->k < m->cap) {
            const int64_t o = m->slot0 + m->k;
            orc_gfeatures(m->bl, m->bu, centre, side, &w->com[3 * c], w->M[c], &w->Q[6 * c],
                          w->count[c], w->next[c] == c + 1, m->eps, &m->feat[10 * o]);
            m->label[o] = group_label(w, c, m->g0, m->g1, dg2);
            m->node[o] = (int32_t)c;
            ++m->k;
        }
        if (w->next[c] != c + 1)
            gsample_walk(m, c);
    }
}

/* Training pairs of the groups of G consecutive sorted ranks of [t0, t1)
 * (group q holds [t0 + qG, min(t0 + qG + G, t1))): per group up to cap kept
 * candidates in pre-order at slot q*cap.. of feat (10 features each),
 * label, node; cnt[q]. */
void orc_group_samples(const int32_t *level, const uint64_t *hkey, const int32_t *begin,
                       const int32_t *count, const int32_t *next, const double *M,
                       const double *com, const double *Q, const double *spos,
                       const double *smass, const double *lo, double L, int64_t t0, int64_t t1,
                       double eps, double theta_lo, double theta_max, double keep, uint64_t seed,
                       int64_t G, int64_t cap, double *feat, double *label, int32_t *node,
                       int64_t *cnt)
{
    const int64_t n = t1;
    const int64_t ng = (t1 - t0 + G - 1) / G;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < ng; ++q) {
        gsample_ctx m;
        memset(&m, 0, sizeof(m));
        m.w = (walk_ctx){level, begin, count, next, M, com, Q, spos, smass, L, 0.0, eps * eps, 2};
        m.hkey = hkey;
        m.lo = lo;
        m.tlo2 = theta_lo * theta_lo;
        m.tmax2 = theta_max * theta_max;
        m.eps = eps;
        m.keep = keep;
        m.seed = seed;
        m.g0 = t0 + q * G;
        m.g1 = m.g0 + G < n ? m.g0 + G : n;
        m.cap = cap;
        m.slot0 = q * cap;
        m.feat = feat;
        m.label = label;
        m.node = node;
        for (int a = 0; a < 3; ++a) {
            m.bl[a] = INFINITY;
            m.bu[a] = -INFINITY;
        }
        for (int64_t i = m.g0; i < m.g1; ++i)
            for (int a = 0; a < 3; ++a) {
                m.bl[a] = fmin(m.bl[a], spos[3 * i + a]);
                m.bu[a] = fmax(m.bu[a], spos[3 * i + a]);
            }
        for (int a = 0; a < 3; ++a) {
            m.bc[a] = 0.5 * (m.bl[a] + m.bu[a]);
            m.bh[a] = 0.5 * (m.bu[a] - m.bl[a]);
        }
        if (next[0] != 1)
            gsample_walk(&m, 0);
        cnt[q] = m.k;
    }
}
