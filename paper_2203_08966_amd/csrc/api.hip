// C ABI of the gfx950 Barnes-Hut library: argument checks (host, before any
// GPU work), object lifetimes, and dispatch to the kernels.
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "bh_internal.h"
#include "mlp.h"

namespace bh {

static thread_local std::string g_err;

int set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// The context of the calling entry point (set by use_device): its
// allocator serves the buffers that grow during the call.
static thread_local const bh_ctx *g_cur = nullptr;

void free_buf(DevBuf &b) {
    if (b.p) {
        if (b.ffree) b.ffree(b.p, b.cap, b.fdev, b.fstream, b.fuser);
        else hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    b.ffree = nullptr;
}

int grow(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 64;
    if (b.cap >= bytes) return BH_OK;
    free_buf(b);
    const size_t want = bytes + bytes / 8 + 256;
    void *p = nullptr;
    const bh_ctx *c = g_cur;
    if (c && c->alloc) {
        p = c->alloc(want, c->device, (void *)c->stream, c->alloc_user);
        if (!p)
            return set_error(BH_E_NOMEM, "caller's allocator refused " + std::to_string(want) +
                                             " bytes");
        b.ffree = c->free_fn;
        b.fuser = c->alloc_user;
        b.fdev = c->device;
        b.fstream = (void *)c->stream;
    } else if (hipMalloc(&p, want) != hipSuccess || !p) {
        hipGetLastError();
        return set_error(BH_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.p = p;
    b.cap = want;
    return BH_OK;
}

int check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(BH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return BH_OK;
}

static int use_device(bh_ctx *c) {
    g_cur = c;
    if (hipSetDevice(c->device) != hipSuccess) {
        hipGetLastError();
        return set_error(BH_E_DEVICE, "hipSetDevice failed");
    }
    return BH_OK;
}

static void free_tree_bufs(bh_tree *t) {
    DevBuf *all[] = {&t->keys_a, &t->keys_b, &t->idx_a, &t->idx_b, &t->spos, &t->smass,
                     &t->bodies, &t->anchors, &t->delta, &t->nstart, &t->offs, &t->hkey,
                     &t->level, &t->begin, &t->count, &t->next, &t->parent, &t->cmask,
                     &t->lvl_list, &t->cx, &t->cy, &t->cz, &t->mom, &t->recs,
                     &t->cube, &t->part, &t->hist, &t->status, &t->misc, &t->cnt_scratch,
                     &t->kc, &t->anorm, &t->est_acc, &t->kids, &t->ulist, &t->mv, &t->s3, &t->oct, &t->wq, &t->gorder,
                     &t->gfb};
    for (DevBuf *b : all) free_buf(*b);
}

static void free_sim(SimState *s) {
    DevBuf *all[] = {&s->pos, &s->vel, &s->mass, &s->acc, &s->phi, &s->id,
                     &s->pos2, &s->vel2, &s->mass2, &s->id2, &s->red, &s->acc_tmp,
                     &s->cnt_pp, &s->cnt_pc, &s->cnt_pq, &s->cnt_sum};
    for (DevBuf *b : all) free_buf(*b);
}

static bool bad_dtype(int d) { return d != BH_F32 && d != BH_F64; }
static size_t dsize(int d) { return d == BH_F32 ? 4 : 8; }

static int check_opts(const bh_force_opts &o, int64_t n) {
    if (o.order != 0 && o.order != BH_ORDER_MIXED && o.order != 2 && o.order != 3)
        return set_error(BH_E_INVALID, "opts.order must be 0, 1 (BH_ORDER_MIXED), 2 or 3");
    if (o.order == BH_ORDER_MIXED && o.mac != BH_MAC_BUDGET)
        return set_error(BH_E_INVALID, "opts.order BH_ORDER_MIXED runs with BH_MAC_BUDGET only");
    if (o.order == 3 && o.mac != BH_MAC_THETA)
        return set_error(BH_E_INVALID, "opts.order 3 (octopole) runs with the opening angle "
                                       "BH_MAC_THETA only");
    if (o.mac == BH_MAC_MLP && o.order != 2)
        return set_error(BH_E_INVALID, "BH_MAC_MLP runs in the quadrupole walk (opts.order 2)");
    if (o.mac != BH_MAC_THETA && o.mac != BH_MAC_MLP && o.mac != BH_MAC_BUDGET &&
        o.mac != BH_MAC_THETA_GUARD)
        return set_error(BH_E_INVALID, "opts.mac must be BH_MAC_THETA, BH_MAC_MLP, BH_MAC_BUDGET "
                                       "or BH_MAC_THETA_GUARD");
    if (o.mac == BH_MAC_THETA_GUARD && o.walk != BH_WALK_BODY)
        return set_error(BH_E_INVALID, "BH_MAC_THETA_GUARD is a per-body walk criterion "
                                       "(group walks open every cell that meets the group)");
    if (o.target_end > 0 &&
        (o.target_begin < 0 || o.target_begin > o.target_end || o.target_end > n))
        return set_error(BH_E_INVALID, "opts target range outside [0, n]");
    if (o.mac != BH_MAC_THETA && o.mac != BH_MAC_THETA_GUARD &&
        !(o.mlp_theta_max > 0 && isfinite(o.mlp_theta_max) && isfinite(o.mlp_log10_tau) &&
          o.mlp_theta_est >= 0 && isfinite(o.mlp_theta_est) && o.mlp_acc_floor >= 0 &&
          isfinite(o.mlp_acc_floor) &&
          (o.mlp_precision == BH_MLP_BF16 || o.mlp_precision == BH_MLP_FP16)))
        return set_error(BH_E_INVALID, "opts learned-criterion parameters invalid");
    if (o.walk != BH_WALK_BODY && o.walk != BH_WALK_GROUP && o.walk != BH_WALK_DIRECT)
        return set_error(BH_E_INVALID,
                         "opts.walk must be BH_WALK_BODY, BH_WALK_GROUP or BH_WALK_DIRECT");
    if (o.walk_stack < 0 || o.walk_stack > 640)
        return set_error(BH_E_INVALID, "opts.walk_stack must be in [0, 640]");
    if (o.walk_cap < 0) return set_error(BH_E_INVALID, "opts.walk_cap must be >= 0");
    return BH_OK;
}

static int check_params(double theta, double eps) {
    if (!(theta >= 0) || !isfinite(theta)) return set_error(BH_E_INVALID, "theta must be finite and >= 0");
    if (!(eps >= 0) || !isfinite(eps)) return set_error(BH_E_INVALID, "eps must be finite and >= 0");
    return BH_OK;
}

static int check_build_args(const void *pos, const void *mass, int dtype, int64_t n, int leaf) {
    if (!pos || !mass) return set_error(BH_E_INVALID, "null pos or mass");
    if (bad_dtype(dtype)) return set_error(BH_E_INVALID, "dtype must be BH_F32 or BH_F64");
    if (n < 1 || n > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "n must be in [1, 2^31 - 2^16]");
    if (leaf < 1 || leaf > kMaxLeaf) return set_error(BH_E_INVALID, "leaf_size must be in [1, 256]");
    // node indices are int32: the cells of one level partition the bodies
    // and at most n / (B + 1) of them are split, so a tree holds at most
    // n leaves plus kLevels * floor(n / (B + 1)) internal cells
    if (n + (int64_t)kLevels * (n / (leaf + 1)) > (int64_t)0x7fffffff)
        return set_error(BH_E_INVALID, "n too large for this leaf_size: the node count could "
                                       "exceed 2^31 - 1 (need n + 21 floor(n / (B + 1)) < 2^31)");
    return BH_OK;
}

}  // namespace bh

using namespace bh;

extern "C" {

const char *bh_version(void) { return "bh-gfx950 0.1"; }

const char *bh_last_error(void) { return g_err.c_str(); }

void bh_force_opts_default(bh_force_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->order = 2;
    o->mac = BH_MAC_THETA;
    o->mlp_theta_max = 1.0;
    o->mlp_log10_tau = -3.0;
    o->mlp_acc_norm = nullptr;
    o->mlp_theta_est = 0.8;
    o->mlp_acc_floor = 0.0;
    o->mlp_precision = BH_MLP_BF16;
    o->walk = BH_WALK_BODY;
    o->walk_stack = 0;
    o->walk_cap = 0;
}

int bh_ctx_create(int device, void *stream, bh_ctx **out) {
    if (!out) return set_error(BH_E_INVALID, "null out");
    *out = nullptr;
    if (device < 0) return set_error(BH_E_INVALID, "device must be >= 0");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        hipGetLastError();
        return set_error(BH_E_DEVICE, "no HIP device available");
    }
    if (device >= count) return set_error(BH_E_INVALID, "device index out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return set_error(BH_E_DEVICE, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(BH_E_DEVICE, std::string("library is built for gfx950, device is ") +
                                          prop.gcnArchName);
    bh_ctx *c = new bh_ctx;
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (use_device(c) || hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return set_error(BH_E_DEVICE, "pinned staging allocation failed");
    }
    // the device address of the allocation-free entry points' fixed scratch
    if (int rc = static_scratch_init(device)) {
        hipHostFree(c->pinned);
        delete c;
        return rc;
    }
    *out = c;
    return BH_OK;
}

int bh_ctx_set_stream(bh_ctx *c, void *stream) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    c->stream = (hipStream_t)stream;
    return BH_OK;
}

int bh_ctx_set_curve(bh_ctx *c, int curve) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (curve != BH_CURVE_MORTON && curve != BH_CURVE_HILBERT)
        return set_error(BH_E_INVALID, "curve must be BH_CURVE_MORTON or BH_CURVE_HILBERT");
    c->curve = curve;
    return BH_OK;
}

int bh_ctx_set_sort(bh_ctx *c, int mode) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (mode != BH_SORT_ADAPTIVE && mode != BH_SORT_FULL)
        return set_error(BH_E_INVALID, "sort mode must be BH_SORT_ADAPTIVE or BH_SORT_FULL");
    c->sort_mode = mode;
    return BH_OK;
}

int bh_ctx_set_allocator(bh_ctx *c, bh_alloc_fn alloc, bh_free_fn free_fn, void *user) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if ((alloc == nullptr) != (free_fn == nullptr))
        return set_error(BH_E_INVALID, "give both allocator functions or neither");
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->alloc_user = user;
    return BH_OK;
}

int bh_ctx_destroy(bh_ctx *c) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (c->live_trees > 0) return set_error(BH_E_STATE, "free the context's trees first");
    use_device(c);
    hipStreamSynchronize(c->stream);
    if (c->sim) {
        free_sim(c->sim);
        delete c->sim;
    }
    if (c->sim_tree) {
        free_tree_bufs(c->sim_tree);
        delete c->sim_tree;
    }
    free_buf(c->mlp_w);
    free_buf(c->mlp_master);
    free_buf(c->mlp_scratch);
    free_buf(c->mlp_gpart);
    free_buf(c->scratch);
    free_buf(c->su_work);
    for (hipEvent_t e : c->events) hipEventDestroy(e);
    if (c->pinned) hipHostFree(c->pinned);
    delete c;
    return BH_OK;
}

int bh_sync(bh_ctx *c) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (use_device(c)) return BH_E_DEVICE;
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_error(BH_E_DEVICE, std::string("device error: ") + hipGetErrorString(e));
    return check_launch("sync");
}

int bh_build(bh_ctx *c, const void *pos, const void *mass, int dtype, int64_t n, int leaf,
             bh_tree **tree) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!tree) return set_error(BH_E_INVALID, "null tree handle");
    int rc = check_build_args(pos, mass, dtype, n, leaf);
    if (rc) return rc;
    if (*tree && (*tree)->ctx != c) return set_error(BH_E_INVALID, "tree belongs to another context");
    if (*tree && *tree == c->sim_tree) return set_error(BH_E_INVALID, "cannot rebuild the simulation tree");
    if (use_device(c)) return BH_E_DEVICE;
    bh_tree *t = *tree;
    const bool fresh = t == nullptr;
    if (fresh) {
        t = new bh_tree;
        t->ctx = c;
    }
    rc = build_tree(c, t, c->curve, pos, mass, dtype, n, leaf, nullptr, nullptr, nullptr, nullptr,
                    nullptr, nullptr, false);
    if (rc) {
        if (fresh) {
            free_tree_bufs(t);
            delete t;
        }
        return rc;
    }
    if (fresh) {
        c->live_trees++;
        *tree = t;
    }
    return BH_OK;
}

int bh_tree_free(bh_tree *t) {
    if (!t) return set_error(BH_E_INVALID, "null tree");
    if (t->ctx && t == t->ctx->sim_tree) return set_error(BH_E_INVALID, "the simulation tree is owned by its context");
    if (t->ctx) {
        use_device(t->ctx);
        hipStreamSynchronize(t->ctx->stream);
        t->ctx->live_trees--;
    }
    free_tree_bufs(t);
    delete t;
    return BH_OK;
}

int bh_forces(bh_tree *t, double theta, double eps, void *acc, const bh_force_opts *opts) {
    if (!t) return set_error(BH_E_INVALID, "null tree");
    if (!acc) return set_error(BH_E_INVALID, "null acc");
    int rc = check_params(theta, eps);
    if (rc) return rc;
    bh_force_opts o;
    if (opts) o = *opts;
    else bh_force_opts_default(&o);
    if ((rc = check_opts(o, t->n))) return rc;
    if (o.walk == BH_WALK_DIRECT)
        return set_error(BH_E_INVALID,
                         "BH_WALK_DIRECT is a simulation mode (bh_sim_init); bh_direct sums "
                         "for given targets");
    // the learned criterion without a network: the plain opening angle at theta
    if (o.mac == BH_MAC_MLP && !t->ctx->mlp_loaded) o.mac = BH_MAC_THETA;
    if (use_device(t->ctx)) return BH_E_DEVICE;
    return run_walk(t, theta, eps, acc, o.phi, o.n_pp, o.n_pc, o, false);
}

int bh_tree_info_get(const bh_tree *t, bh_tree_info *info) {
    if (!t || !info) return set_error(BH_E_INVALID, "null tree or info");
    if (use_device(t->ctx)) return BH_E_DEVICE;
    memset(info, 0, sizeof(*info));
    info->n = t->n;
    info->m = t->m;
    info->depth = (int32_t)t->depth;
    info->dtype = t->dtype;
    info->leaf_size = t->leaf;
    info->last_mac = t->last_mac;
    info->curve = t->curve;
    info->movers = t->movers;
    for (int d = 0; d < 3; ++d) info->lo[d] = t->lo[d];
    info->side = t->L;
    return BH_OK;
}

int bh_tree_export(const bh_tree *t, uint64_t *keys, uint32_t *perm, uint64_t *hkey,
                   int32_t *level, int32_t *begin, int32_t *count, int32_t *next,
                   int32_t *parent, int32_t *cmask, double *mass, double *com, double *quad) {
    if (!t) return set_error(BH_E_INVALID, "null tree");
    if (use_device(t->ctx)) return BH_E_DEVICE;
    if (hipStreamSynchronize(t->ctx->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "device error before export");
    const size_t n = (size_t)t->n, m = (size_t)t->m;
    bool ok = true;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (dst && ok) ok = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
    };
    cp(keys, t->sorted_keys, 8 * n);
    cp(perm, t->perm, 4 * n);
    cp(hkey, t->hkey.p, 8 * m);
    cp(level, t->level.p, 4 * m);
    cp(begin, t->begin.p, 4 * m);
    cp(count, t->count.p, 4 * m);
    cp(next, t->next.p, 4 * m);
    cp(parent, t->parent.p, 4 * m);
    cp(cmask, t->cmask.p, 4 * m);
    if (ok && (mass || com || quad)) {
        std::vector<Moments> mom(m);
        std::vector<int32_t> c3(3 * m);
        cp(mom.data(), t->mom.p, sizeof(Moments) * m);
        cp(c3.data(), t->cx.p, 4 * m);
        cp(c3.data() + m, t->cy.p, 4 * m);
        cp(c3.data() + 2 * m, t->cz.p, 4 * m);
        if (ok) {
            const double h = ldexp(t->L, -(kLevels + 1));
            for (size_t i = 0; i < m; ++i) {
                const Moments &q = mom[i];
                if (mass) mass[i] = q.m;
                if (com)
                    for (int d = 0; d < 3; ++d)
                        com[3 * i + d] = t->lo[d] + c3[d * m + i] * h + q.c[d];
                if (quad) {
                    const double tr = q.t[0] + q.t[3] + q.t[5];
                    quad[6 * i + 0] = 3 * q.t[0] - tr;
                    quad[6 * i + 1] = 3 * q.t[1];
                    quad[6 * i + 2] = 3 * q.t[2];
                    quad[6 * i + 3] = 3 * q.t[3] - tr;
                    quad[6 * i + 4] = 3 * q.t[4];
                    quad[6 * i + 5] = 3 * q.t[5] - tr;
                }
            }
        }
    }
    if (!ok) {
        hipGetLastError();
        return set_error(BH_E_DEVICE, "tree export copy failed");
    }
    return BH_OK;
}

// ---------------------------------------------------------------- simulation
// Forces of the current (just rebuilt) step.  The accelerations of the
// previous step are still in s->acc, in the order the tree was built from,
// and give the learned criterion its |a_i|.  The potential is computed when
// asked for (the initial walk; bh_energy): a step's loop body needs only the
// accelerations.
static int sim_forces(bh_ctx *c, bool want_phi) {
    SimState *s = c->sim;
    int rc;
    if (s->opts.walk == BH_WALK_DIRECT) {  // every pair, no tree (Sec. 3, direct method)
        if (c->walk_ev) hipEventRecord(c->walk_ev[0], c->stream);
        rc = launch_direct_all(c->stream, s->dtype, s->n, s->pos.p, s->mass.p, s->eps,
                               s->acc.p, s->phi.p, c->scratch);
        if (c->walk_ev) hipEventRecord(c->walk_ev[1], c->stream);
        s->phi_valid = rc == BH_OK;
        return rc;
    }
    // a recorded step (bh_sim_timing) also counts its interactions
    const bool count = c->walk_ev != nullptr && s->cnt_sum.p != nullptr;
    uint32_t *npp = count ? (uint32_t *)s->cnt_pp.p : nullptr;
    uint32_t *npc = count ? (uint32_t *)s->cnt_pc.p : nullptr;
    bh_force_opts wo = s->opts;
    wo.n_pq = count ? (uint32_t *)s->cnt_pq.p : nullptr;
    rc = run_walk(c->sim_tree, s->theta, s->eps, s->acc.p, want_phi ? s->phi.p : nullptr,
                  npp, npc, wo, true, s->have_acc ? s->acc.p : nullptr);
    s->phi_valid = want_phi && rc == BH_OK;
    s->counted = rc == BH_OK && count;
    return rc;
}

static int sim_rebuild(bh_ctx *c, const void *pos, const void *vel, const void *mass,
                       const uint32_t *id, bool presorted) {
    SimState *s = c->sim;
    int rc = build_tree(c, c->sim_tree, s->curve, pos, mass, s->dtype, s->n, s->leaf, vel, id,
                        s->pos2.p, s->vel2.p, s->mass2.p, (uint32_t *)s->id2.p, presorted);
    if (rc) return rc;
    std::swap(s->pos, s->pos2);
    std::swap(s->vel, s->vel2);
    std::swap(s->mass, s->mass2);
    std::swap(s->id, s->id2);
    return BH_OK;
}

int bh_sim_init(bh_ctx *c, const void *pos, const void *vel, const void *mass, int dtype,
                int64_t n, int leaf, double theta, double eps, const bh_force_opts *opts) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!vel) return set_error(BH_E_INVALID, "null vel");
    int rc = check_build_args(pos, mass, dtype, n, leaf);
    if (rc) return rc;
    if ((rc = check_params(theta, eps))) return rc;
    bh_force_opts o;
    if (opts) o = *opts;
    else bh_force_opts_default(&o);
    o.phi = nullptr;
    o.n_pp = o.n_pc = nullptr;
    o.target_begin = o.target_end = 0;
    o.mlp_acc_norm = nullptr;  // the previous step's accelerations serve instead
    if ((rc = check_opts(o, n))) return rc;
    // the learned criterion without a network: the plain opening angle at theta
    if (o.mac == BH_MAC_MLP && !c->mlp_loaded) o.mac = BH_MAC_THETA;
    if (use_device(c)) return BH_E_DEVICE;
    if (!c->sim) c->sim = new SimState;
    if (!c->sim_tree) {
        c->sim_tree = new bh_tree;
        c->sim_tree->ctx = c;
    }
    // a new simulation starts without the previous one's group-walk
    // fallback predictions (its walks then depend on its inputs alone)
    c->sim_tree->gfb_ng = -1;
    SimState *s = c->sim;
    s->dtype = dtype;
    s->n = n;
    s->leaf = leaf;
    s->curve = c->curve;
    s->theta = theta;
    s->eps = eps;
    s->opts = o;
    s->opts.n_pq = nullptr;  // a recorded step counts into the state's own buffers
    s->have_acc = false;
    const size_t e = dsize(dtype);
    if ((rc = grow(s->pos, 3 * e * n)) || (rc = grow(s->vel, 3 * e * n)) ||
        (rc = grow(s->mass, e * n)) || (rc = grow(s->acc, 3 * e * n)) ||
        (rc = grow(s->phi, e * n)) || (rc = grow(s->id, 4ull * n)) ||
        (rc = grow(s->pos2, 3 * e * n)) || (rc = grow(s->vel2, 3 * e * n)) ||
        (rc = grow(s->mass2, e * n)) || (rc = grow(s->id2, 4ull * n)) ||
        (rc = grow(s->red, 8ull * (2 * 1024 + 8))))
        return rc;
    // first build gathers straight from the caller's arrays
    if ((rc = sim_rebuild(c, pos, vel, mass, nullptr, false))) return rc;
    if ((rc = sim_forces(c, true))) return rc;
    s->have_acc = true;
    return BH_OK;
}

static constexpr int64_t kMaxTimedSteps = 65536;

static hipEvent_t *step_events(bh_ctx *c) {
    if (!c->timing || c->timed_steps >= kMaxTimedSteps) return nullptr;
    const size_t need = 7 * (size_t)(c->timed_steps + 1);
    while (c->events.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    return &c->events[7 * (size_t)c->timed_steps];
}

int bh_leapfrog_step(bh_ctx *c, double dt) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    if (!isfinite(dt)) return set_error(BH_E_INVALID, "dt must be finite");
    if (use_device(c)) return BH_E_DEVICE;
    SimState *s = c->sim;
    hipEvent_t *ev = step_events(c);
    auto mark = [&](int k) {
        if (ev) hipEventRecord(ev[k], c->stream);
    };
    int rc;
    mark(0);
    // kick (dt/2) and drift (dt)
    if ((rc = launch_kick_drift(c->stream, s->dtype, s->n, s->pos.p, s->vel.p, s->acc.p,
                                0.5 * dt, dt)))
        return rc;
    mark(1);
    // new tree and accelerations at the drifted positions (the direct method
    // keeps the bodies in the order of the first build and needs no tree)
    if (s->opts.walk != BH_WALK_DIRECT &&
        (rc = sim_rebuild(c, s->pos.p, s->vel.p, s->mass.p, (const uint32_t *)s->id.p, true)))
        return rc;
    mark(2);
    c->walk_ev = ev ? ev + 5 : nullptr;  // the walk kernel alone: events 5, 6
    rc = sim_forces(c, false);
    c->walk_ev = nullptr;
    if (rc) return rc;
    mark(3);
    // second kick (dt/2)
    rc = launch_kick(c->stream, s->dtype, s->n, s->vel.p, s->acc.p, 0.5 * dt);
    mark(4);
    if (ev) c->timed_steps++;
    if (rc == BH_OK && s->counted) {  // after the step's last event: not in its phases
        s->counted = false;
        rc = launch_count_sum(c->stream, s->n, (const uint32_t *)s->cnt_pp.p,
                              (const uint32_t *)s->cnt_pc.p, (const uint32_t *)s->cnt_pq.p,
                              (unsigned long long *)s->cnt_sum.p);
    }
    return rc;
}

int bh_sim_timing(bh_ctx *c, int enable) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (enable && c->sim && c->sim->opts.walk != BH_WALK_DIRECT) {
        // per-body counts and their running sums for the recorded steps
        SimState *s = c->sim;
        if (use_device(c)) return BH_E_DEVICE;
        int rc;
        if ((rc = grow(s->cnt_pp, 4ull * s->n)) || (rc = grow(s->cnt_pc, 4ull * s->n)) ||
            (rc = grow(s->cnt_pq, 4ull * s->n)) || (rc = grow(s->cnt_sum, 24)))
            return rc;
        if (hipMemsetAsync(s->cnt_sum.p, 0, 24, c->stream) != hipSuccess)
            return set_error(BH_E_DEVICE, "clearing the interaction counters failed");
    }
    c->timing = enable != 0;
    if (enable) c->timed_steps = 0;
    return BH_OK;
}

int bh_sim_counts_get(bh_ctx *c, int64_t *pp, int64_t *pc) {
    if (!c || !pp || !pc) return set_error(BH_E_INVALID, "null argument");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    SimState *s = c->sim;
    *pp = *pc = 0;
    if (!s->cnt_sum.p) return BH_OK;  // nothing recorded (or the direct method)
    if (use_device(c)) return BH_E_DEVICE;
    unsigned long long h[2] = {0, 0};
    if (hipMemcpyAsync(h, s->cnt_sum.p, 16, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "reading the interaction counters failed");
    *pp = (int64_t)h[0];
    *pc = (int64_t)h[1];
    return BH_OK;
}

int bh_sim_counts_pq_get(bh_ctx *c, int64_t *pq) {
    if (!c || !pq) return set_error(BH_E_INVALID, "null argument");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    SimState *s = c->sim;
    *pq = 0;
    if (!s->cnt_sum.p) return BH_OK;  // nothing recorded (or the direct method)
    if (use_device(c)) return BH_E_DEVICE;
    unsigned long long h = 0;
    if (hipMemcpyAsync(&h, (const char *)s->cnt_sum.p + 16, 8, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "reading the interaction counters failed");
    *pq = (int64_t)h;
    return BH_OK;
}

int bh_sim_timing_get(bh_ctx *c, double *ms, int64_t *steps) {
    if (!c || !ms || !steps) return set_error(BH_E_INVALID, "null argument");
    if (use_device(c)) return BH_E_DEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "device error while timing");
    for (int k = 0; k < 5; ++k) ms[k] = 0.0;
    for (int64_t s = 0; s < c->timed_steps; ++s) {
        hipEvent_t *e = &c->events[7 * (size_t)s];
        for (int k = 0; k < 5; ++k) {
            float t = 0.f;
            const int a = k < 4 ? k : 5;  // ms[4]: events 5 .. 6
            if (hipEventElapsedTime(&t, e[a], e[a + 1]) != hipSuccess)
                return set_error(BH_E_DEVICE, "hipEventElapsedTime failed");
            ms[k] += t;
        }
    }
    *steps = c->timed_steps;
    return BH_OK;
}

int bh_sim_get(bh_ctx *c, void *pos, void *vel, void *acc) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    if (use_device(c)) return BH_E_DEVICE;
    SimState *s = c->sim;
    int rc = BH_OK;
    const uint32_t *id = (const uint32_t *)s->id.p;
    if (pos && (rc = launch_unpermute(c->stream, s->dtype, s->n, id, s->pos.p, pos))) return rc;
    if (vel && (rc = launch_unpermute(c->stream, s->dtype, s->n, id, s->vel.p, vel))) return rc;
    if (acc && (rc = launch_unpermute(c->stream, s->dtype, s->n, id, s->acc.p, acc))) return rc;
    return BH_OK;
}

int bh_energy(bh_ctx *c, double *ekin, double *epot) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!ekin || !epot) return set_error(BH_E_INVALID, "null output");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    if (use_device(c)) return BH_E_DEVICE;
    SimState *s = c->sim;
    int rc;
    if (!s->phi_valid) {
        // the potential of the current state: the same walk (tree, theta,
        // criterion; |a_i| from the current accelerations) with phi, its
        // accelerations set aside
        if ((rc = grow(s->acc_tmp, 3 * dsize(s->dtype) * s->n))) return rc;
        if ((rc = run_walk(c->sim_tree, s->theta, s->eps, s->acc_tmp.p, s->phi.p, nullptr,
                           nullptr, s->opts, true, s->acc.p)))
            return rc;
        s->phi_valid = true;
    }
    double *red = (double *)s->red.p;
    rc = launch_energy(c->stream, s->dtype, s->n, s->vel.p, s->mass.p, s->phi.p, red,
                           red + 2 * 1024);
    if (rc) return rc;
    double *hp = (double *)c->pinned + 64;
    if (hipMemcpyAsync(hp, red + 2 * 1024, 16, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "energy copy failed");
    *ekin = hp[0];
    *epot = hp[1];
    return BH_OK;
}

int bh_sim_tree(bh_ctx *c, bh_tree **tree) {
    if (!c || !tree) return set_error(BH_E_INVALID, "null argument");
    if (!c->sim || !c->sim->have_acc) return set_error(BH_E_STATE, "bh_sim_init has not run");
    *tree = c->sim_tree;
    return BH_OK;
}

int bh_direct(bh_ctx *c, const void *pos, const void *mass, int dtype, int64_t n,
              const int64_t *targets, int64_t nt, double eps, double *acc, double *phi) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!pos || !mass || !targets || !acc) return set_error(BH_E_INVALID, "null pointer");
    if (bad_dtype(dtype)) return set_error(BH_E_INVALID, "dtype must be BH_F32 or BH_F64");
    if (n < 1 || n > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "n out of range");
    if (nt < 1 || nt > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "nt out of range");
    if (!(eps >= 0) || !isfinite(eps)) return set_error(BH_E_INVALID, "eps must be finite and >= 0");
    if (use_device(c)) return BH_E_DEVICE;
    return launch_direct(c->stream, dtype, n, pos, mass, targets, nt, eps, acc, phi, c->scratch);
}

int bh_direct_static(bh_ctx *c, const void *pos, const void *mass, int dtype, int64_t n,
                     const int64_t *targets, int64_t nt, double eps, double *acc, double *phi) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!pos || !mass || !targets || !acc) return set_error(BH_E_INVALID, "null pointer");
    if (bad_dtype(dtype)) return set_error(BH_E_INVALID, "dtype must be BH_F32 or BH_F64");
    if (n < 1 || n > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "n out of range");
    if (nt < 1 || nt > direct_static_max_targets())
        return set_error(BH_E_INVALID, "nt out of range: 1 .. 524288 targets per call");
    if (!(eps >= 0) || !isfinite(eps)) return set_error(BH_E_INVALID, "eps must be finite and >= 0");
    if (use_device(c)) return BH_E_DEVICE;
    return launch_direct_static(c->stream, c->device, dtype, n, pos, mass, targets, nt, eps, acc,
                                phi);
}

int bh_standard_units(bh_ctx *c, void *pos, void *vel, void *mass, int dtype, int64_t n,
                      double *stats) {
    if (!c) return set_error(BH_E_INVALID, "null ctx");
    if (!pos || !vel || !mass) return set_error(BH_E_INVALID, "null pointer");
    if (bad_dtype(dtype)) return set_error(BH_E_INVALID, "dtype must be BH_F32 or BH_F64");
    if (n < 2 || n > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "n must be in [2, 2^31 - 2^16]");
    if (use_device(c)) return BH_E_DEVICE;
    double *hp = (double *)c->pinned + 128;
    int rc = standard_units(c->stream, dtype, n, pos, vel, mass, c->scratch, c->su_work, hp);
    if (rc) return rc;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "standard units: device error");
    if (stats)
        for (int k = 0; k < 3; ++k) stats[k] = hp[k];
    return BH_OK;
}

// ---------------------------------------------------------------- learned criterion
int bh_mlp_set(bh_ctx *c, const double *params) {
    if (!c || !params) return set_error(BH_E_INVALID, "null argument");
    for (int k = 0; k < kMlpParams; ++k)
        if (!isfinite(params[k])) return set_error(BH_E_INVALID, "non-finite parameter");
    if (use_device(c)) return BH_E_DEVICE;
    int rc = grow(c->mlp_master, 3ull * 4 * kMlpParams);
    if (rc) return rc;
    std::vector<float> h(3 * kMlpParams, 0.f);
    for (int k = 0; k < kMlpParams; ++k) h[k] = (float)params[k];
    if (hipMemcpyAsync(c->mlp_master.p, h.data(), h.size() * 4, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "parameter upload failed");
    c->mlp_step = 0;
    return mlp_pack(c);
}

int bh_mlp_get(bh_ctx *c, double *params) {
    if (!c || !params) return set_error(BH_E_INVALID, "null argument");
    if (!c->mlp_loaded) return set_error(BH_E_STATE, "no parameters loaded");
    if (use_device(c)) return BH_E_DEVICE;
    std::vector<float> h(kMlpParams);
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(h.data(), c->mlp_master.p, 4 * kMlpParams, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(BH_E_DEVICE, "parameter copy failed");
    for (int k = 0; k < kMlpParams; ++k) params[k] = h[k];
    return BH_OK;
}

int bh_mlp_samples(bh_tree *t, double eps, double theta_lo, double theta_max, double keep,
                   uint64_t seed, int64_t capacity, float *feat, float *label, int32_t *node,
                   int32_t *body, int64_t *total) {
    if (!t || !total) return set_error(BH_E_INVALID, "null argument");
    if (t->dtype != BH_F64) return set_error(BH_E_INVALID, "training pairs need a BH_F64 tree");
    if (!(theta_lo >= 0) || !(theta_max > theta_lo) || !isfinite(theta_max) || !(eps >= 0) ||
        !isfinite(eps) || !(keep >= 0 && keep <= 1))
        return set_error(BH_E_INVALID, "bad band, eps or keep");
    if (feat && (!label || !node || !body || capacity < 0))
        return set_error(BH_E_INVALID, "null output");
    if (use_device(t->ctx)) return BH_E_DEVICE;
    return mlp_samples(t, eps, theta_lo, theta_max, keep, seed, capacity, feat, label, node, body,
                       total);
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int bh_mlp_train(bh_ctx *c, const float *feat, const float *label, int64_t n,
                 const bh_mlp_train_cfg *cfg, double *loss) {
    if (!c || !feat || !label || !cfg) return set_error(BH_E_INVALID, "null argument");
    if (n < 1 || n > (int64_t)0x7fffffff) return set_error(BH_E_INVALID, "n out of range");
    if (cfg->epochs < 0 || cfg->batch < 1 || !(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) ||
        !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0) ||
        !(cfg->quantile >= 0 && cfg->quantile < 1))
        return set_error(BH_E_INVALID, "bad training configuration");
    if (!c->mlp_loaded) return set_error(BH_E_STATE, "set initial parameters first");
    if (use_device(c)) return BH_E_DEVICE;
    const MlpTrainCfg tc{(float)cfg->lr, (float)cfg->beta1, (float)cfg->beta2, (float)cfg->eps,
                         (float)cfg->quantile};
    int rc = grow(c->mlp_scratch, 64);
    if (rc) return rc;
    float *lacc = (float *)c->mlp_scratch.p;
    const int bs_max = (int)(cfg->batch < n ? cfg->batch : n);
    for (int e = 0; e < cfg->epochs; ++e) {
        // this epoch's order: j -> (a j + b) mod n with gcd(a, n) = 1
        uint64_t h = cfg->seed * 0x9E3779B97F4A7C15ull + (uint64_t)e * 0xD1B54A32D192ED03ull;
        uint64_t a = (h % (uint64_t)n) | 1u;
        while (gcd_u64(a, (uint64_t)n) != 1) a = (a + 2) % (uint64_t)n | 1u;
        const uint64_t b = (h >> 17) % (uint64_t)n;
        hipMemsetAsync(lacc, 0, 4, c->stream);
        for (int64_t base = 0; base < n; base += bs_max) {
            const int bs = (int)(n - base < bs_max ? n - base : bs_max);
            if ((rc = mlp_grad_step(c, feat, label, n, base, bs, a, b, nullptr, lacc, true,
                                    ++c->mlp_step, tc)))
                return rc;
        }
        if (loss) {
            float lv = 0.f;
            if (hipMemcpyAsync(&lv, lacc, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess)
                return set_error(BH_E_DEVICE, "loss copy failed");
            loss[e] = (double)lv / (double)n;
        }
    }
    return mlp_pack(c);
}

int bh_mlp_grad(bh_ctx *c, const float *feat, const float *label, int64_t n, double quantile,
                float *grad, double *loss) {
    if (!c || !feat || !label || !grad) return set_error(BH_E_INVALID, "null argument");
    if (n < 1 || n > (1 << 24)) return set_error(BH_E_INVALID, "n out of range");
    if (!(quantile >= 0 && quantile < 1)) return set_error(BH_E_INVALID, "quantile out of range");
    if (!c->mlp_loaded) return set_error(BH_E_STATE, "no parameters loaded");
    if (use_device(c)) return BH_E_DEVICE;
    int rc = grow(c->mlp_scratch, 64);
    if (rc) return rc;
    float *lacc = (float *)c->mlp_scratch.p;
    hipMemsetAsync(lacc, 0, 4, c->stream);
    const MlpTrainCfg tc{1.f, 0.9f, 0.999f, 1e-8f, (float)quantile};
    if ((rc = mlp_grad_step(c, feat, label, n, 0, (int)n, 1, 0, grad, lacc, false, 1, tc)))
        return rc;
    float lv = 0.f;
    if (hipMemcpyAsync(&lv, lacc, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return set_error(BH_E_DEVICE, "loss copy failed");
    if (loss) *loss = (double)lv / (double)n;
    return BH_OK;
}

int bh_mlp_infer(bh_ctx *c, const float *feat, int64_t n, int precision, float *pred) {
    if (!c || !feat || !pred) return set_error(BH_E_INVALID, "null argument");
    if (n < 1 || n > (int64_t)0x7fff0000) return set_error(BH_E_INVALID, "n out of range");
    if (precision != BH_MLP_BF16 && precision != BH_MLP_FP16)
        return set_error(BH_E_INVALID, "precision must be BH_MLP_BF16 or BH_MLP_FP16");
    if (!c->mlp_loaded) return set_error(BH_E_STATE, "no parameters loaded");
    if (use_device(c)) return BH_E_DEVICE;
    return mlp_infer(c, feat, n, precision, pred);
}

}  // extern "C"
