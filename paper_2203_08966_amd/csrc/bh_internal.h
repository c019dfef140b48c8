// Internal declarations of the gfx950 Barnes-Hut library (HIP, wave64).
// Device data layouts, launch helpers and the host-side objects behind the
// opaque handles of bh.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "bh.h"

namespace bh {

constexpr int kLevels = 21;        // key bits per dimension (Sec. 4.4)
constexpr int kMaxLeaf = 256;      // largest supported leaf capacity B
constexpr int kThreads = 256;      // default block size (4 waves)

// Root cube, device resident: lower corner and side (a power of two).
struct Cube {
    double lo[3];
    double L;
};

// FP64 cell moments from the upward pass: total mass, centre of mass
// relative to the cell centre, and the raw second moment
// sum m (y - com)(y - com)^T about the COM (xx xy xz yy yz zz).
struct Moments {
    double m;
    double c[3];
    double t[6];
};

// Walk record of one cell, FP32: 64 bytes, read with uniform (scalar) loads.
// Centre as (integer centre in units of h = L 2^-22) * h, relative to the
// root corner: an integer below 2^23 times a power of two, so exact in FP32,
// and the difference of two such centres is exact too.  COM and quadrupole
// relative to that centre; traceless quadrupole as 5 components.
struct alignas(64) NodeRec32 {
    float cx, cy, cz;
    float mx, my, mz;
    float m;
    float qxx, qxy, qxz, qyy, qyz;
    int begin, count, next;
    float l2;  // side^2
};

// FP64 walk record (128 bytes).
struct alignas(128) NodeRec64 {
    double cx, cy, cz;
    int level, pad2;
    int begin, count, next, pad0;
    double mx, my, mz, m;
    double qxx, qxy, qxz, qyy, qyz;
    double l2;  // side^2
};

template <typename R> struct NodeRecT;
template <> struct NodeRecT<float> { using type = NodeRec32; };
template <> struct NodeRecT<double> { using type = NodeRec64; };

// Body record for the walk: offset from its leaf's centre and mass.
template <typename R> struct alignas(4 * sizeof(R)) BodyRec {
    R x, y, z, m;
};

// A body's anchor: its leaf's centre, scaled like NodeRec centres, and the
// leaf's node index.
template <typename R> struct alignas(4 * sizeof(R)) Anchor {
    R x, y, z;
    int leaf;
};

// Grow-only device buffer.
// Its memory comes from the caller's allocator when the owning context has
// one (the free function and its arguments are kept with the buffer).
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    bh_free_fn ffree = nullptr;
    void *fuser = nullptr;
    int fdev = 0;
    void *fstream = nullptr;
};

struct SimState;

}  // namespace bh

// Opaque handles.
struct bh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t epoch = 0;              // look-back epoch of the radix sort
    void *pinned = nullptr;          // small pinned host staging area
    bh::SimState *sim = nullptr;
    bh_tree *sim_tree = nullptr;
    int live_trees = 0;
    int curve = BH_CURVE_MORTON;     // space-filling curve of later builds
    int sort_mode = BH_SORT_ADAPTIVE;  // re-sort of a simulation's rebuilds
    // learned acceptance criterion
    bh::DevBuf mlp_w;                // packed inference weights (MlpPacked)
    bh::DevBuf mlp_master;           // FP32 parameters, Adam m, Adam v
    bh::DevBuf mlp_scratch, mlp_gpart;
    int mlp_loaded = 0;
    int mlp_step = 0;                // Adam steps taken
    int mlp_version = 0;             // bumped whenever the parameters change
    bh_alloc_fn alloc = nullptr;     // caller's allocator (NULL: hipMalloc)
    bh_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    bh::DevBuf scratch;              // direct-sum partials
    bh::DevBuf su_work;              // standard units: FP64 acc, phi, partials
    // phase timing of simulation steps
    bool timing = false;
    std::vector<hipEvent_t> events;  // 7 per recorded step
    int64_t timed_steps = 0;
    hipEvent_t *walk_ev = nullptr;   // set during a timed step: around the walk kernel
};

struct bh_tree {
    bh_ctx *ctx = nullptr;
    int dtype = BH_F32;
    int64_t n = 0, m = 0;
    int leaf = 1;
    int depth = 0;
    int32_t lvl_cnt[22] = {}, lvl_base[22] = {};  // cells per level, first slot in lvl_list
    int last_mac = -1;  // criterion the last walk of this tree used (-1: none yet)
    int curve = BH_CURVE_MORTON;  // the curve the bodies are sorted along
    bool resort_ok = false;       // the last build completed (its keys and leaves are valid)
    int64_t movers = -1;          // bodies the last build's re-sort moved (-1: full sort)
    double lo[3] = {0, 0, 0}, L = 1.0;
    // body-indexed
    bh::DevBuf keys_a, keys_b, idx_a, idx_b;  // radix-sort ping-pong
    bh::DevBuf spos, smass;                    // sorted positions and masses (dtype)
    bh::DevBuf bodies, anchors;                // walk body records, leaf centres
    bh::DevBuf delta, nstart, offs;            // topology scratch
    // node-indexed
    bh::DevBuf hkey, level, begin, count, next, parent, cmask, lvl_list;
    bh::DevBuf cx, cy, cz;
    bh::DevBuf mom, recs;
    // small scratch
    bh::DevBuf cube, part, hist, status, misc, cnt_scratch;
    // error budget: M l^3 per cell; |a| per sorted rank; estimate
    // accelerations
    bh::DevBuf kc, anorm, est_acc;
    bh::DevBuf kids;                           // group walk: children per node
    bh::DevBuf ulist;                          // upward pass: subtree roots, upper cells
    bh::DevBuf mv;                             // re-sort: the movers' keys and positions
    bh::DevBuf s3, oct;                        // order 3: raw third moments, octopole records
    int64_t oct_tree_id = -1;
    bh::DevBuf wq;                             // group walk: queue counters
    bh::DevBuf gorder;                         // group walk: work items in hand-out order
    bh::DevBuf gfb;                            // group walk: per-group fallback prediction
    uint64_t gfb_sig = 0;                      //   parameters it was made with
    int64_t gfb_ng = -1;                       //   and group count
    int64_t kids_tree_id = -1;
    int64_t build_id = 0, kc_tree_id = -1;
    uint64_t *sorted_keys = nullptr;           // result buffers after the sort
    uint32_t *perm = nullptr;
};

namespace bh {

struct SimState {
    int dtype = BH_F32;
    int64_t n = 0;
    int leaf = 16;
    int curve = BH_CURVE_MORTON;               // every rebuild's curve, fixed at init
    double theta = 0.5, eps = 0.0;
    bh_force_opts opts{};
    DevBuf pos, vel, mass, acc, phi, id;       // key order (current)
    DevBuf pos2, vel2, mass2, id2;             // gather targets
    DevBuf red;                                // energy reduction scratch
    DevBuf acc_tmp;                            // accelerations of an energy walk
    DevBuf cnt_pp, cnt_pc, cnt_pq, cnt_sum;    // interaction counts of recorded steps
    bool have_acc = false;
    bool phi_valid = false;                    // phi belongs to the current state
    bool counted = false;                      // cnt_pp/cnt_pc hold this step's counts
};

// ---- host helpers (api.hip)
int set_error(int code, const std::string &msg);
int grow(DevBuf &b, size_t bytes);
void free_buf(DevBuf &b);
int check_launch(const char *what);

// ---- tree construction (build.hip)
// Builds the tree from device pos/mass of `dtype`.  If `vel`/`id` are given
// (simulation), they are permuted alongside into vel_out/id_out.
// presorted: the bodies come in the order of this tree's previous build (a
// simulation step), which allows the nearly sorted re-sort
int build_tree(bh_ctx *ctx, bh_tree *t, int curve, const void *pos, const void *mass,
               int dtype, int64_t n, int leaf, const void *vel, const uint32_t *id,
               void *pos_out, void *vel_out, void *mass_out, uint32_t *id_out, bool presorted);

// Octopole records of the tree (order-3 walks), computed on first use per
// build: 8 values of the tree's dtype per node (see build.hip).
int ensure_octopole(bh_tree *t);

// ---- walk (walk.hip)
// prev_acc: accelerations in the tree's input order from an earlier step;
// the learned criterion takes |a_i| from it unless opts give norms.
int run_walk(bh_tree *t, double theta, double eps, void *acc, void *phi, uint32_t *npp,
             uint32_t *npc, const bh_force_opts &o, bool sorted_out,
             const void *prev_acc = nullptr);

// ---- simulation helpers (sim.hip)
int launch_kick(hipStream_t s, int dtype, int64_t n, void *vel, const void *acc, double h);
int launch_kick_drift(hipStream_t s, int dtype, int64_t n, void *pos, void *vel,
                      const void *acc, double h, double dt);
int launch_energy(hipStream_t s, int dtype, int64_t n, const void *vel, const void *mass,
                  const void *phi, double *red, double *host_out2);
int launch_unpermute(hipStream_t s, int dtype, int64_t n, const uint32_t *id, const void *src,
                     void *dst);
// out[0] += sum a, out[1] += sum b, out[2] += sum c (n values each)
int launch_count_sum(hipStream_t s, int64_t n, const uint32_t *a, const uint32_t *b,
                     const uint32_t *c, unsigned long long *out);
int launch_direct(hipStream_t s, int dtype, int64_t n, const void *pos, const void *mass,
                  const int64_t *targets, int64_t nt, double eps, double *acc, double *phi,
                  DevBuf &scratch);
// The direct sum with its partial sums in a fixed device array of
// kStaticScratchBytes (no allocation).  static_scratch_init takes the
// array's address on `device` (the current device) once; calls that
// overlap on one GPU share the array and race.
constexpr size_t kStaticScratchBytes = 16ull << 20;
int static_scratch_init(int device);
int64_t direct_static_max_targets();
int launch_direct_static(hipStream_t s, int device, int dtype, int64_t n, const void *pos,
                         const void *mass, const int64_t *targets, int64_t nt, double eps,
                         double *acc, double *phi);
// every body of (pos, mass) as target, arithmetic and outputs in dtype
int launch_direct_all(hipStream_t s, int dtype, int64_t n, const void *pos, const void *mass,
                      double eps, void *acc, void *phi, DevBuf &scratch);
// in place; synchronous.  host (pinned, 8 doubles) returns E_kin, E_pot
// and the total mass before the scaling.
int standard_units(hipStream_t s, int dtype, int64_t n, void *pos, void *vel, void *mass,
                   DevBuf &scratch, DevBuf &work, double *host);

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace bh
