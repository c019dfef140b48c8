/*
 * bh.h -- C ABI of the MI355X (gfx950) Barnes-Hut library.
 *
 * The operations follow the Barnes-Hut loop body of Brandt, "On Distributed
 * Gravitational N-Body Simulations" (arXiv:2203.08966), Sec. 3: build the
 * octree over the bodies, compute each cell's mass distribution bottom-up,
 * walk the tree per body with the opening-angle test side/distance < theta,
 * then integrate with the kick-drift-kick leapfrog of Sec. 2.3.
 *
 * Conventions shared by every entry point:
 *  - Units: G = 1 (Sec. 2.2).
 *  - Pointers named "device" are device memory on the context's GPU; "host"
 *    pointers are ordinary CPU memory.  Positions, velocities and
 *    accelerations are N x 3, row-major, contiguous (x0 y0 z0 x1 ...);
 *    masses are N.  Element type is given by a dtype argument (BH_F32 or
 *    BH_F64); accelerations and potentials come back in the tree's dtype.
 *  - The caller owns every pointer it passes.  The library never keeps a
 *    caller pointer after a call returns; trees and simulation state live in
 *    library-owned device memory freed by bh_tree_free / bh_ctx_destroy.
 *  - All GPU work is enqueued on the context's stream; calls return without
 *    waiting unless stated.  bh_build waits once for the node count.
 *  - Every call returns BH_OK (0) or a negative status.  Argument checks run
 *    on the host before any GPU work, so a rejected call has no effect.
 *    Asynchronous device failures surface from bh_sync or the next call.
 *    bh_last_error() gives a message for the calling thread's last failure.
 *  - Results are deterministic: identical inputs and options give bitwise
 *    identical outputs on every run.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef BH_H
#define BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BH_OK = 0,
    BH_E_INVALID = -1,   /* bad argument (null pointer, size, parameter, dtype) */
    BH_E_NOMEM = -2,     /* device allocation failed */
    BH_E_DEVICE = -3,    /* HIP runtime / kernel failure, or no usable GPU */
    BH_E_STATE = -4,     /* call out of order (e.g. step before bh_sim_init) */
    BH_E_NONFINITE = -5  /* a position is NaN or infinite */
};

enum { BH_F32 = 0, BH_F64 = 1 };

/* How the walk takes its decisions. */
enum {
    BH_WALK_BODY = 0, /* per body, as in Sec. 3 (wavefronts share the sweep) */
    BH_WALK_GROUP = 1, /* one decision per cell for each group of
                         BH_GROUP_BODIES consecutive sorted bodies (one
                         wavefront, one lane per body), against the distance
                         from the cell's COM to the group's bounding box; a
                         cell whose cube meets the box is always opened */
    BH_WALK_DIRECT = 2 /* simulation only (bh_sim_init): no tree, every pair
                          summed directly, the direct method of Sec. 3, in
                          the simulation's dtype (each tile of 256 sources
                          summed into FP64); O(N^2).  theta, the criterion and the
                          order are ignored; bh_forces rejects it. */
};

/* Bodies per group of BH_WALK_GROUP: groups start at target_begin. */
enum { BH_GROUP_BODIES = 64 };

/* Acceptance criterion used by the walk. */
enum {
    BH_MAC_THETA = 0,  /* side/distance < theta (Sec. 3) */
    BH_MAC_MLP = 1,    /* learned: the network's predicted error of the
                          particle-cell term below tau |a_i| (per group and
                          cell; see bh_mlp_set) */
    BH_MAC_BUDGET = 2, /* error budget: M l^3 / d^5 < tau |a_i| (no network) */
    BH_MAC_THETA_GUARD = 3 /* side/distance < theta and the body outside the
                              cell's closed cube (a containment guard; not in
                              the paper; BH_WALK_BODY only).  Below theta =
                              1/sqrt(3) it equals BH_MAC_THETA. */
};

/* Space-filling curve the bodies are sorted along (bh_ctx_set_curve). */
enum {
    BH_CURVE_MORTON = 0,  /* Morton (Z) order, Sec. 4.4 (default) */
    BH_CURVE_HILBERT = 1  /* Peano-Hilbert order, the remedy Sec. 4.4 names
                             for the Morton order's jumps (a variant) */
};

/* How a simulation step's rebuild sorts its bodies (bh_ctx_set_sort). */
enum {
    BH_SORT_ADAPTIVE = 0, /* default: the bodies arrive in the previous
                             build's order, nearly sorted after a short step
                             (Sec. 4.4); only the bodies that left their
                             leaf's key range (and the leaves whose bodies
                             fell out of order) are radix-sorted, then merged
                             with the rest.  Same result as BH_SORT_FULL. */
    BH_SORT_FULL = 1      /* always the full 8-pass radix sort */
};

/* Arithmetic of the network's inference (MFMA operands; FP32 accumulate). */
enum {
    BH_MLP_BF16 = 0,
    BH_MLP_FP16 = 1
};

typedef struct bh_ctx bh_ctx;
typedef struct bh_tree bh_tree;

/* Mixed expansion order of the error budget (opts.order with BH_MAC_BUDGET):
 * per cell the monopole term where M side^3 + (7/2) |Q|_F d < tau |a| d^5,
 * else the quadrupole term where M side^3 < tau |a| d^5, else the cell is
 * opened (both kinds of term meet the budget; a quadrupole term costs less
 * than opening the cell). */
enum { BH_ORDER_MIXED = 1 };

/* Options of a force evaluation.  Fill with bh_force_opts_default first. */
typedef struct {
    int order;        /* 0: monopole only; 2: monopole + quadrupole (default);
                         3: and the octopole, the l = 3 term of Sec. 2.2
                         (BH_MAC_THETA only; its moments are computed from
                         the tree on the first order-3 walk of a build);
                         BH_ORDER_MIXED (1): BH_MAC_BUDGET only */
    int mac;          /* BH_MAC_THETA (default), BH_MAC_MLP, BH_MAC_BUDGET or
                         BH_MAC_THETA_GUARD */
    void *phi;        /* optional device out, N values in caller order: the
                         potential at each body from the same walk */
    uint32_t *n_pp;   /* optional device out, N: particle-particle count */
    uint32_t *n_pc;   /* optional device out, N: particle-cell count */
    int64_t target_begin; /* walk only bodies of sorted rank [begin, end); */
    int64_t target_end;   /* end <= 0 means all.  Outputs of other bodies are
                             left untouched. */
    /* BH_MAC_BUDGET (FP32 walk of order 2 or 0): accept a multi-body cell
     * iff side/d < mlp_theta_max, the body is outside it, and
     * M side^3 < 10^mlp_log10_tau |a_i| d^5 (per group: d_g and the
     * smallest |a_i|); with order 0 (monopole terms) the left side also
     * holds (7/2) |Q|_F d, d^-4 times which bounds the quadrupole term the
     * cell drops (Sec. 2.2), Q its traceless quadrupole.  BH_MAC_MLP (FP32
     * quadrupole walk only): the learned decision described with
     * bh_mlp_set, with tau = 10^mlp_log10_tau; with no network loaded the
     * walk takes the opening-angle test at theta instead.  |a_i| comes from
     * mlp_acc_norm (device, n norms in the tree's dtype, caller order) or,
     * if NULL, from a monopole walk at mlp_theta_est run first (a
     * simulation step uses the previous step's accelerations instead). */
    double mlp_theta_max;     /* default 1.0 */
    double mlp_log10_tau;     /* default -3 */
    const void *mlp_acc_norm; /* default NULL */
    double mlp_theta_est;     /* default 0.8 */
    int walk;                 /* BH_WALK_BODY (default), BH_WALK_GROUP or
                                 BH_WALK_DIRECT (simulation only) */
    int walk_stack;           /* group walk: LDS stack entries per wavefront,
                                 1..640, 0 = 640; subtrees that do not fit
                                 are walked without the stack (same result) */
    int walk_cap;             /* group walk: a group whose work (particle-cell
                                 terms + particle-particle bodies, per body)
                                 would exceed this is walked per body with the
                                 same criterion; 0 = 6144 (4096 with
                                 BH_MAC_BUDGET).  A group (of one
                                 run) that did is walked per body straight
                                 away in the next walks of the same tree
                                 object with the same parameters and targets,
                                 also after the tree is rebuilt in place: 15
                                 walks, or, when a walk has more than 4 groups
                                 per wavefront it launches, 1 walk after a
                                 first excess, doubling with each repeated
                                 excess up to 15 (a group walk that fits
                                 starts it over).  A simulation step may then
                                 walk such a group per body although it would
                                 now fit. */
    double mlp_acc_floor;     /* BH_MAC_MLP / BH_MAC_BUDGET: |a_i| in the test
                                 is replaced by max(|a_i|, f <|a|>), f this
                                 value (>= 0) and <|a|> the mean of the n
                                 norms, so that bodies where the field nearly
                                 cancels do not force near-direct sums; the
                                 budget then bounds the error relative to the
                                 larger of the body's and f times the mean
                                 acceleration.  Default 0 (none). */
    int mlp_precision;        /* BH_MAC_MLP: BH_MLP_BF16 (default) or
                                 BH_MLP_FP16 operands of the network */
    uint32_t *n_pq;           /* optional device out, N: of the particle-cell
                                 terms, those with the quadrupole (all of
                                 them at order 2 or 3, none at order 0) */
} bh_force_opts;

/* Library version string. */
const char *bh_version(void);

/* Message for the calling thread's most recent failed call ("" if none). */
const char *bh_last_error(void);

void bh_force_opts_default(bh_force_opts *opts);

/* Create a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the null stream).  *out receives the context.
 * BH_E_DEVICE when the device cannot be used. */
int bh_ctx_create(int device, void *stream, bh_ctx **out);
int bh_ctx_set_stream(bh_ctx *ctx, void *stream);

/* The curve that later builds of this context (bh_build, bh_sim_init) sort
 * the bodies along.  A simulation keeps the curve of its bh_sim_init for
 * every rebuild of its steps, whatever this is set to later.  BH_CURVE_HILBERT: the
 * 63-bit key is the Peano-Hilbert index of the same 21-bit integer point
 * (Butz's construction: axis x in bit 0 of each level's three bits; the
 * curve starts at the cube's corner lo).  A prefix of k octal digits of
 * either key names the same level-k cube, so the tree has the same cells:
 * only the order of bodies, of a cell's children and of the nodes (still
 * pre-order) changes.  Cells keep their Morton hashed keys and child masks
 * by octant.  BH_E_INVALID for another value. */
int bh_ctx_set_curve(bh_ctx *ctx, int curve);

/* The sort of later simulation rebuilds on this context: BH_SORT_ADAPTIVE
 * (default) or BH_SORT_FULL.  Both give the stable sort of the keys (ties in
 * input order), bit for bit; the adaptive one falls back to the full sort
 * when more than a quarter of the bodies move.  bh_build always sorts in
 * full.  An adaptive rebuild waits for the device once more (to size the
 * movers' sort).  BH_E_INVALID for another value. */
int bh_ctx_set_sort(bh_ctx *ctx, int mode);

/* Device memory from the caller's allocator (e.g. a framework's caching
 * allocator) instead of hipMalloc.  alloc(bytes, device, stream, user)
 * returns device memory of at least `bytes` on `device`, usable in the
 * order of `stream` (the context's stream at the time), aligned to at
 * least 16 bytes (the kernels use 16-byte vector accesses), or NULL (the call
 * then fails with BH_E_NOMEM); free_fn(ptr, bytes, device, stream, user)
 * takes back a block with the arguments of its allocation.  Both or
 * neither (NULL, NULL: hipMalloc again).  Buffers allocated earlier keep
 * the allocator they came from.  Every device buffer of the context, its
 * trees and its simulation state grows through it; the library frees a
 * buffer only when it grows it or when its owner is freed, so the
 * functions must stay valid until the context is destroyed. */
typedef void *(*bh_alloc_fn)(size_t bytes, int device, void *stream, void *user);
typedef void (*bh_free_fn)(void *ptr, size_t bytes, int device, void *stream, void *user);
int bh_ctx_set_allocator(bh_ctx *ctx, bh_alloc_fn alloc, bh_free_fn free_fn, void *user);
/* Frees the context, its simulation state and its learned-criterion
 * weights.  Trees built with it must be freed first. */
int bh_ctx_destroy(bh_ctx *ctx);
/* Waits for the context's stream; reports asynchronous device errors. */
int bh_sync(bh_ctx *ctx);

/* ---------------------------------------------------------------------
 * bh_build -- octree construction (Sec. 3 build step; Sec. 4.4 Morton keys,
 * Sec. 4.2 pre-order serialisation, Sec. 4.7 hashed keys).
 *
 * pos: device, n x 3 of dtype; mass: device, n of dtype (>= 0).
 * leaf_size B in [1, 256]: a cell holding more than B bodies is split in
 * half in each dimension, down to key level 21; only non-empty children
 * exist (B = 1 is the paper's tree).  The root is the smallest power-of-two
 * cube holding every body with its corner on a multiple of half its side;
 * keys are 21 bits per dimension, x more significant than y than z.
 * Bodies are sorted by key, ties in input order.  Nodes are stored in
 * pre-order.  Cell moments (mass, centre of mass, quadrupole about it) are
 * computed in FP64 whatever the dtype.
 *
 * *tree: NULL to allocate a new tree, or an existing tree of this context
 * to rebuild into (its memory is reused and grown as needed).
 * Errors: BH_E_INVALID (null pointer, n < 1, n > 2^31 - 2^16, n +
 * 21 floor(n / (B + 1)) >= 2^31 (the bound on the node count), leaf_size
 * out of range, bad dtype), BH_E_NONFINITE, BH_E_NOMEM, BH_E_DEVICE.  Waits for the
 * device once (to size the node arrays).
 * ------------------------------------------------------------------- */
int bh_build(bh_ctx *ctx, const void *pos, const void *mass, int dtype, int64_t n,
             int leaf_size, bh_tree **tree);
int bh_tree_free(bh_tree *tree);

/* ---------------------------------------------------------------------
 * bh_forces -- per-body tree walk (Sec. 3, "Compute Cell Force").
 *
 * For every body: starting below the root, each child cell C in octant
 * order contributes particle-particle if it holds one body; a particle-cell
 * term with its multipole expansion if side^2 < theta^2 * d^2 (d from the
 * body to C's centre of mass); particle-particle with each of its bodies if
 * it is a leaf; otherwise C is opened.  Softening eps applies to every term
 * (s^2 = r^2 + eps^2).  The self pair is skipped.  Arithmetic is the tree's
 * dtype; the FP32 walk takes every position relative to a cell centre.
 *
 * acc: device out, n x 3 of the tree's dtype, caller order.
 * theta >= 0, eps >= 0, finite.  opts NULL = defaults.  BH_MAC_MLP with no
 * network loaded (bh_mlp_set) falls back to the opening angle at theta
 * (BH_MAC_THETA, same walk kind); bh_tree_info_get reports which criterion
 * ran.  Errors: BH_E_INVALID, BH_E_DEVICE.
 * ------------------------------------------------------------------- */
int bh_forces(bh_tree *tree, double theta, double eps, void *acc, const bh_force_opts *opts);

/* Tree shape: n bodies, m nodes, depth, root cube (lo, side), dtype, leaf
 * size, curve, and the criterion (BH_MAC_*) the tree's last walk used, -1 before
 * the first: BH_MAC_THETA after a BH_MAC_MLP request with no network
 * loaded (the fallback to the plain opening angle). */
typedef struct {
    int64_t n, m;
    int32_t depth, dtype, leaf_size, last_mac;
    int32_t curve, reserved; /* BH_CURVE_* the bodies are sorted along */
    double lo[3], side;
    int64_t movers;          /* bodies the last build's adaptive re-sort moved;
                                -1 when it sorted in full */
} bh_tree_info;
int bh_tree_info_get(const bh_tree *tree, bh_tree_info *info);

/* Copies the tree to host buffers (any may be NULL): sorted keys[n],
 * perm[n] (caller index of each sorted rank), and per node in pre-order:
 * hkey[m] (1 << 3k | Morton key prefix, whatever the curve), level[m], begin[m] (first sorted rank),
 * count[m], next[m] (first node after the subtree), parent[m] (-1 root),
 * cmask[m] (bit d set iff child octant d exists), mass[m], com[m x 3]
 * (absolute), quad[m x 6] (xx xy xz yy yz zz, sum m(3 y_a y_b - |y|^2 d_ab)
 * about the COM).  Synchronous. */
int bh_tree_export(const bh_tree *tree, uint64_t *keys, uint32_t *perm, uint64_t *hkey,
                   int32_t *level, int32_t *begin, int32_t *count, int32_t *next,
                   int32_t *parent, int32_t *cmask, double *mass, double *com, double *quad);

/* ---------------------------------------------------------------------
 * Simulation: kick-drift-kick leapfrog with a fixed step (Sec. 2.3).
 * bh_sim_init copies pos/vel/mass (device, dtype) into context-owned state,
 * builds the tree and computes the initial accelerations (and potential).
 * Each bh_leapfrog_step(dt) does v += a dt/2; x += v dt; rebuild; walk
 * (accelerations); v += a dt/2.  State is kept in key order between steps.  With
 * BH_MAC_MLP / BH_MAC_BUDGET, opts.mlp_acc_norm is ignored: the initial
 * walk estimates |a_i| by a monopole walk, later steps use the previous
 * step's accelerations.
 * ------------------------------------------------------------------- */
int bh_sim_init(bh_ctx *ctx, const void *pos, const void *vel, const void *mass, int dtype,
                int64_t n, int leaf_size, double theta, double eps, const bh_force_opts *opts);
int bh_leapfrog_step(bh_ctx *ctx, double dt);
/* Copies state to device buffers in caller order (any may be NULL). */
int bh_sim_get(bh_ctx *ctx, void *pos, void *vel, void *acc);
/* Kinetic energy sum m v^2 / 2 and potential energy sum m phi / 2 (each
 * pair once, softened; Sec. 2.4), accumulated in FP64.  Steps compute
 * accelerations only; phi comes from the last walk if it computed it (the
 * initial walk, the direct method, an earlier bh_energy of the same state),
 * else from one more walk of the current tree with the simulation's
 * options (a relative criterion takes |a_i| from the current
 * accelerations), whose accelerations are discarded.  Synchronous. */
int bh_energy(bh_ctx *ctx, double *ekin, double *epot);
/* The simulation's current tree (owned by the context; do not free).  With
 * BH_WALK_DIRECT, the tree of bh_sim_init: the steps build none. */
int bh_sim_tree(bh_ctx *ctx, bh_tree **tree);

/* Per-phase timing of bh_leapfrog_step with HIP events recorded on the
 * context's stream.  enable = 1 clears the totals and starts recording (at
 * most 65536 steps); 0 stops.  bh_sim_timing_get waits for the stream and
 * returns, summed over the recorded steps, the milliseconds spent in
 * ms[0] kick + drift, ms[1] tree build, ms[2] walk (with its set-up
 * kernels), ms[3] final kick, ms[4] the walk kernel alone (ms holds 5
 * values), and the number of steps.  A recorded tree-walk step also counts
 * its interactions (the walk kernel then writes per-body counts, 8 bytes a
 * body more); bh_sim_counts_get waits for the stream and returns the sums
 * of the particle-particle and particle-cell counts over the walks of the
 * steps recorded since timing was last enabled (0 for the direct method or
 * when nothing was recorded). */
int bh_sim_timing(bh_ctx *ctx, int enable);
int bh_sim_timing_get(bh_ctx *ctx, double *ms, int64_t *steps);
int bh_sim_counts_get(bh_ctx *ctx, int64_t *n_pp, int64_t *n_pc);
/* Of the recorded steps' particle-cell terms, those with the quadrupole (as
 * opts.n_pq counts them). */
int bh_sim_counts_pq_get(bh_ctx *ctx, int64_t *n_pq);

/* ---------------------------------------------------------------------
 * bh_direct -- FP64 direct summation (Sec. 2.1) for a subset of targets,
 * the reference for the tree's error.  pos/mass: device, dtype; targets: device
 * int64[nt] caller indices; acc: device f64 nt x 3; phi: device f64 nt or
 * NULL.  Self pair skipped.
 * ------------------------------------------------------------------- */
int bh_direct(bh_ctx *ctx, const void *pos, const void *mass, int dtype, int64_t n,
              const int64_t *targets, int64_t nt, double eps, double *acc, double *phi);

/* ---------------------------------------------------------------------
 * bh_direct_static -- bh_direct for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results bitwise identical to
 * bh_direct's.  It allocates nothing: the partial sums go to a fixed
 * 16 MiB array in each GPU's global memory, held from the first
 * bh_ctx_create on that GPU until the process ends, which limits a call to
 * nt <= 524288 targets (larger nt: BH_E_INVALID, nothing launched).  Every
 * call on one GPU shares that array: calls that overlap on one GPU (other
 * streams, other contexts or threads) race and give wrong results.  The
 * array needs no clearing between calls: each call writes every partial it
 * reads.
 * ------------------------------------------------------------------- */
int bh_direct_static(bh_ctx *ctx, const void *pos, const void *mass, int dtype, int64_t n,
                     const int64_t *targets, int64_t nt, double eps, double *acc, double *phi);

/* ---------------------------------------------------------------------
 * bh_standard_units -- scale a system in place to the standard units of
 * Sec. 2.4: masses to total 1, positions and velocities to the
 * centre-of-mass frame, velocities by one factor so that E_kin = -E_pot/2,
 * then lengths by b and velocities by 1/sqrt(b) so that the total energy is
 * -1/4.  E_pot is the unsoftened direct sum (FP64, every pair: O(N^2)).
 * pos, vel: device n x 3, mass: device n, all of dtype.  stats: optional
 * host double[3] out: E_kin, E_pot and total mass before the scaling (after
 * the shift).  Synchronous.  Fails with BH_E_INVALID if the total mass or
 * the kinetic energy is not positive, BH_E_NONFINITE on non-finite sums
 * (e.g. two bodies at one point).
 * ------------------------------------------------------------------- */
int bh_standard_units(bh_ctx *ctx, void *pos, void *vel, void *mass, int dtype, int64_t n,
                      double *stats);

/* ---------------------------------------------------------------------
 * Learned acceptance criterion (not in the paper; it stands in for the
 * opening-angle test of Sec. 3).
 *
 * One decision per (group, cell): a network 10 -> 32 (ReLU) -> 32 (ReLU)
 * -> 1 predicts log10 of the largest error the cell's quadrupole
 * particle-cell term makes on the group's bodies, in units of the error
 * budget's model M side^3 / d_g^5 (d_g: distance from the cell's COM to the
 * box): a coefficient k_C per group and cell.  The walk accepts the cell
 * for the whole group iff its cube misses the box, side < mlp_theta_max d_g,
 * and
 *     pred + log10(M side^3 / d_g^5) < log10(tau a_min),
 * a_min the group's smallest (floored) |a_i|; a group walked per body takes
 * the same decision with each body as its own group (box of zero extent),
 * and so does BH_WALK_BODY.  Inside the walk the network runs on MFMA
 * (bf16, or fp16 with BH_MLP_FP16; FP32 sums), one 64-row batch per round of
 * candidate cells, one per lane.  Parameters (BH_MLP_PARAMS doubles, host):
 * W1[32][10] b1[32] W2[32][32] b2[32] w3[32] b3, held on the device as FP32
 * master weights with Adam state and packed to bf16 and fp16 operands.
 * Features (l side, d_c distance from the COM to the box centre, h the
 * box's half-diagonal, n the unit vector from the box centre to the COM,
 * g = COM - cell centre, Q the traceless quadrupole):
 * log2(l/d_g) in [-8, 8], min(log2(d_c/d_g), 8), h/(h + d_g),
 * n.Q.n/(M l^2), |Q|_F/(M l^2), g.n/l, |g|/l, log2(count)/21,
 * min(eps/d_g, 1), leaf (0/1).
 * ------------------------------------------------------------------- */
#define BH_MLP_PARAMS 1441

/* Load parameters (host, FP64 values rounded to FP32); resets Adam. */
int bh_mlp_set(bh_ctx *ctx, const double *params);
/* Copy the current FP32 parameters to host doubles. */
int bh_mlp_get(bh_ctx *ctx, double *params);

/* Training pairs from a BH_F64 tree: the bodies in sorted order form
 * groups of BH_GROUP_BODIES; each group walks the tree leaving alone the
 * cells whose cube misses its box with side < theta_lo d_g and opening all
 * others; every multi-body cell whose cube misses the box with
 * theta_lo d_g <= side < theta_max d_g is a candidate, kept iff the
 * SplitMix64 hash of (seed ^ (first rank << 32 | node)) >> 11 is below
 * keep * 2^53.  Kept pairs are written densely, by group then pre-order:
 * feat (device f32, the pair's 10 features), label (device f32:
 * log10(max_i |a_pc,i - a_exact,i| d_g^5 / (M side^3)) over the group's bodies with
 * a_exact the direct sum over the cell's bodies, FP64, floored at 1e-12
 * inside), node and the group's first sorted rank (device i32).  *total
 * gets the number of kept pairs; with feat == NULL only *total is computed.
 * BH_E_INVALID if capacity < *total.  Synchronous. */
int bh_mlp_samples(bh_tree *tree, double eps, double theta_lo, double theta_max, double keep,
                   uint64_t seed, int64_t capacity, float *feat, float *label, int32_t *node,
                   int32_t *group, int64_t *total);

typedef struct {
    int epochs;        /* passes over the set */
    int batch;         /* minibatch size (>= 1) */
    double lr, beta1, beta2, eps;  /* Adam */
    uint64_t seed;     /* per-epoch order: sample (a j + c) mod n, a coprime to n */
    double quantile;   /* 0: mean-squared error; q in (0, 1): pinball loss
                          mean(max(q r, (q - 1) r)), r = label - prediction,
                          whose minimiser is the label's q-quantile */
} bh_mlp_train_cfg;

/* Trains the loaded parameters on n pairs (device feat f32 n x 10, label
 * f32 n) with the configured loss and Adam, then packs them for inference.
 * loss (host, optional): mean loss of each epoch.  Synchronous. */
int bh_mlp_train(bh_ctx *ctx, const float *feat, const float *label, int64_t n,
                 const bh_mlp_train_cfg *cfg, double *loss);

/* Gradient (device f32 BH_MLP_PARAMS) and mean loss (host) of the loaded
 * parameters over n pairs as one batch (quantile as in bh_mlp_train_cfg);
 * parameters unchanged. */
int bh_mlp_grad(bh_ctx *ctx, const float *feat, const float *label, int64_t n, double quantile,
                float *grad, double *loss);

/* MFMA inference, 64 rows per wavefront, operands in bf16 or fp16
 * (precision BH_MLP_BF16 / BH_MLP_FP16), FP32 accumulation: pred (device
 * f32 n) for feat (device f32 n x 10). */
int bh_mlp_infer(bh_ctx *ctx, const float *feat, int64_t n, int precision, float *pred);

#ifdef __cplusplus
}
#endif
#endif /* BH_H */
