// Per-body tree walk on gfx950 (Sec. 3, "Compute Cell Force").
//
// One wavefront walks 64 consecutive bodies in key order.  The nodes are in
// pre-order with a skip pointer `next` (first node after the subtree), so the
// union of the 64 recursive walks is one forward sweep over the node array:
//
//   every lane keeps `resume`, the next node index it needs; a lane is
//   active at node idx when resume <= idx.  An active lane takes its own
//   decision for the node exactly as the recursive walk would (one-body cell
//   -> particle-particle; side^2 < theta^2 d^2 -> particle-cell, with the
//   test in the walk's precision; leaf -> particle-particle with its bodies;
//   else open).  A lane that opens the
//   node resumes at idx + 1 (its first child); any other active lane resumes
//   at next[idx].  The wave moves to idx + 1 if any lane opened, else to
//   next[idx]; that is always the smallest resume point of the wave.
//
// Each lane therefore sees exactly its own accepted cells and bodies, in
// pre-order, with no stack, and its arithmetic does not depend on which
// other bodies share its wave.  The node index is wave-uniform, so node
// records and leaf bodies are read with scalar loads and broadcast.
//
// Positions are relative to cell centres: a body is stored as the centre of
// its leaf plus a small offset.  Centres are integers (units h = L 2^-22,
// below 2^23) times h, so the difference of the body's leaf centre and any
// cell centre is exact in FP32; adding the offset is the only rounding.
#include "bh_internal.h"
#include "mlp.h"

namespace bh {
namespace {

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

enum : int { kNone = 0, kPP = 1, kPC = 2, kOpen = 3 };

// Particle-particle terms of the bodies [jb, je) on the lanes in `pp`;
// SELF: some lane's own body may be among them (skipped by index).
// Runs on the lanes that take the particle-particle branch (exec mask).
template <typename R, bool PHI, bool CNT, bool SELF>
__device__ __forceinline__ void leaf_pp(const BodyRec<R> *__restrict__ bodies, int jb, int je,
                                        int i, R X, R Y, R Z, R eps2, R &sx, R &sy, R &sz,
                                        R &sp, uint32_t &cpp) {
    R px = 0, py = 0, pz = 0, pq = 0;
    for (int j = jb; j < je; ++j) {
        const BodyRec<R> s = bodies[j];
        if (!SELF || j != i) {
            const R dx = s.x - X, dy = s.y - Y, dz = s.z - Z;
            R r2 = dx * dx + eps2;
            r2 = dy * dy + r2;
            r2 = dz * dz + r2;
            const R inv = rsq(r2);
            const R minv = s.m * inv;
            const R mi3 = minv * (inv * inv);
            px += mi3 * dx;
            py += mi3 * dy;
            pz += mi3 * dz;
            if (PHI) pq -= minv;
            if (CNT && SELF) ++cpp;
        }
    }
    if (CNT && !SELF) cpp += (uint32_t)(je - jb);
    sx += px;
    sy += py;
    sz += pz;
    if (PHI) sp += pq;
}

// Learned-criterion parameters of a walk: per cell k_C M l^3, per sorted
// rank |a_i|, theta_max^2 and tau.
struct MlpMac {
    const float *kc;
    const float *anorm;
    float tmax2, tau;
};

template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED_OUT, bool MLP>
__global__ __launch_bounds__(256) void k_walk(
    const typename NodeRecT<R>::type *__restrict__ nodes, int m,
    const BodyRec<R> *__restrict__ bodies, const Anchor<R> *__restrict__ anchors,
    const uint32_t *__restrict__ perm, int nbodies, int t0, int t1, int nwaves_padded,
    R theta2, R eps2, R *__restrict__ acc, R *__restrict__ phi_out,
    uint32_t *__restrict__ npp_out, uint32_t *__restrict__ npc_out, MlpMac mac) {
    using Rec = typename NodeRecT<R>::type;
    // XCD-aware placement: consecutive workgroups land on different XCDs,
    // so hand each XCD a contiguous run of 8 logical blocks (spatially
    // close waves then share that XCD's L2).
    const int nblk = nwaves_padded / 4;
    const int b = blockIdx.x;
    const int xcd = b & 7, r = b >> 3;
    const int lb = (r >> 3) * 64 + xcd * 8 + (r & 7);
    if (lb >= nblk) return;
    const int wave = lb * 4 + (int)(threadIdx.x >> 6);
    const int base = t0 + wave * 64;
    if (base >= t1) return;
    const int i = base + (int)lane_id();
    const bool live = i < t1;

    R ox = 0, oy = 0, oz = 0;
    R ax = 0, ay = 0, az = 0;
    int myleaf = -1;
    if (live) {
        const BodyRec<R> me = bodies[i];
        ox = me.x;
        oy = me.y;
        oz = me.z;
        const Anchor<R> an = anchors[i];
        ax = an.x;
        ay = an.y;
        az = an.z;
        myleaf = an.leaf;
    }
    R sx = 0, sy = 0, sz = 0, sp = 0;
    uint32_t cpp = 0, cpc = 0;
    float tau_a = 0.f;  // tau |a_i|
    if (MLP && live) tau_a = mac.tau * mac.anorm[i];

    const bool root_leaf = nodes[0].next == 1;
    int idx = root_leaf ? 0 : 1;
    int resume = live ? idx : 0x7fffffff;

    while (idx < m) {
        idx = uniform(idx);
        const Rec nd = nodes[idx];
        const bool act = resume <= idx;
        const int nxt = uniform(nd.next);
        const int cnt = uniform(nd.count);
        // position relative to the cell centre (the centre difference is exact)
        const R X = (ax - nd.cx) + ox;
        const R Y = (ay - nd.cy) + oy;
        const R Z = (az - nd.cz) + oz;
        bool pp = false, open = false;
        if (cnt == 1 || idx == 0) {
            pp = act;  // one body (or the root leaf): particle-particle
        } else {
            const R x = X - nd.mx, y = Y - nd.my, z = Z - nd.mz;
            const R d2 = x * x + y * y + z * z;
            bool accept;
            if (MLP) {
                // predicted error k_C (l/d)^3 M/d^2 below tau |a_i|, l/d below
                // theta_max, and the body outside the cell
                const float kcv = mac.kc[idx];
                const R hs = (R)0.5 * sqrt(nd.l2);
                const bool inside = fabs(X) <= hs && fabs(Y) <= hs && fabs(Z) <= hs;
                accept = act && nd.l2 < (R)mac.tmax2 * d2 && !inside &&
                         kcv < tau_a * (d2 * d2 * sqrt(d2));
            } else {
                accept = act && nd.l2 < theta2 * d2;
            }
            {
                if (accept) {  // skipped as a whole when no lane accepts
                    const R inv = rsq(d2 + eps2);
                    const R inv2 = inv * inv;
                    const R inv3 = inv * inv2;
                    if (ORDER2) {
                        const R qzz = -nd.qxx - nd.qyy;
                        const R qx = nd.qxx * x + nd.qxy * y + nd.qxz * z;
                        const R qy = nd.qxy * x + nd.qyy * y + nd.qyz * z;
                        const R qz = nd.qxz * x + nd.qyz * y + qzz * z;
                        const R xqx = x * qx + y * qy + z * qz;
                        const R inv5 = inv3 * inv2;
                        const R t5 = xqx * inv5;
                        const R g = nd.m * inv3 + (R)2.5 * t5 * inv2;
                        sx = inv5 * qx + sx;
                        sy = inv5 * qy + sy;
                        sz = inv5 * qz + sz;
                        sx = -g * x + sx;
                        sy = -g * y + sy;
                        sz = -g * z + sz;
                        if (PHI) sp = sp - nd.m * inv - (R)0.5 * t5;
                    } else {
                        const R g = nd.m * inv3;
                        sx = -g * x + sx;
                        sy = -g * y + sy;
                        sz = -g * z + sz;
                        if (PHI) sp = sp - nd.m * inv;
                    }
                    if (CNT) ++cpc;
                }
            }
            if (nxt == idx + 1) pp = act && !accept;  // leaf
            else open = act && !accept;
        }
        if (pp) {
            const int jb = uniform(nd.begin);
            const int je = min(jb + cnt, nbodies);  // guard
            if (myleaf == idx)  // the lane's own leaf: skip itself
                leaf_pp<R, PHI, CNT, true>(bodies, jb, je, i, X, Y, Z, eps2, sx, sy, sz, sp, cpp);
            else
                leaf_pp<R, PHI, CNT, false>(bodies, jb, je, i, X, Y, Z, eps2, sx, sy, sz, sp, cpp);
        }
        const uint64_t any_open = __ballot(open);
        if (act) resume = open ? idx + 1 : nxt;
        idx = any_open ? idx + 1 : (nxt > idx ? nxt : idx + 1);  // always moves forward
    }
    if (live) {
        const int o = SORTED_OUT ? i : (int)perm[i];
        acc[3 * (int64_t)o + 0] = sx;
        acc[3 * (int64_t)o + 1] = sy;
        acc[3 * (int64_t)o + 2] = sz;
        if (PHI) phi_out[o] = sp;
        if (CNT) {
            npp_out[o] = cpp;
            npc_out[o] = cpc;
        }
    }
}

template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED, bool MLP>
void launch(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
            uint32_t *npp, uint32_t *npc, const MlpMac &mac) {
    const int nw = div_up(t1 - t0, 64);
    const int nblk = div_up(nw, 4);
    const int nblk_pad = div_up(nblk, 64) * 64;
    k_walk<R, ORDER2, PHI, CNT, SORTED, MLP><<<nblk_pad, 256, 0, t->ctx->stream>>>(
        (const typename NodeRecT<R>::type *)t->recs.p, (int)t->m,
        (const BodyRec<R> *)t->bodies.p, (const Anchor<R> *)t->anchors.p, t->perm, (int)t->n, t0,
        t1, nblk_pad * 4, (R)(theta * theta), (R)(eps * eps), (R *)acc, (R *)phi, npp, npc, mac);
}

template <typename R, bool ORDER2, bool MLP>
void dispatch2(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
               uint32_t *npp, uint32_t *npc, bool sorted, const MlpMac &mac) {
    const bool P = phi != nullptr, C = npp != nullptr;
#define BH_W(p, c, s) launch<R, ORDER2, p, c, s, MLP>(t, t0, t1, theta, eps, acc, phi, npp, npc, mac)
    if (sorted) {
        if (P) BH_W(true, false, true);
        else BH_W(false, false, true);
    } else if (P && C) BH_W(true, true, false);
    else if (P) BH_W(true, false, false);
    else if (C) BH_W(false, true, false);
    else BH_W(false, false, false);
#undef BH_W
}

}  // namespace

int run_walk(bh_tree *t, double theta, double eps, void *acc, void *phi, uint32_t *npp,
             uint32_t *npc, const bh_force_opts &o, bool sorted_out, const void *prev_acc) {
    int t0 = 0, t1 = (int)t->n;
    if (o.target_end > 0) {
        t0 = (int)o.target_begin;
        t1 = (int)o.target_end;
    }
    if (t1 <= t0) return BH_OK;
    if ((npp != nullptr) != (npc != nullptr)) {  // the kernel writes both or neither
        int rc = grow(t->cnt_scratch, 4ull * t->n);
        if (rc) return rc;
        if (!npp) npp = (uint32_t *)t->cnt_scratch.p;
        else npc = (uint32_t *)t->cnt_scratch.p;
    }
    MlpMac mac{nullptr, nullptr, 0.f, 0.f};
    if (o.mac == BH_MAC_MLP || o.mac == BH_MAC_BUDGET) {
        if (t->dtype != BH_F32 || o.order != 2)
            return set_error(BH_E_INVALID, "the learned criterion runs in the FP32 quadrupole walk");
        int rc = mlp_cells(t, eps, o.mac == BH_MAC_MLP);
        if (rc) return rc;
        if (o.mlp_acc_norm) {
            rc = mlp_anorm(t, nullptr, o.mlp_acc_norm, true);
        } else if (prev_acc) {
            rc = mlp_anorm(t, prev_acc, nullptr, true);
        } else {
            // estimate |a_i| of the targets with a monopole walk at theta_est
            if ((rc = grow(t->est_acc, 12ull * t->n))) return rc;
            bh_force_opts eo;
            bh_force_opts_default(&eo);
            eo.order = 0;
            eo.target_begin = t0;
            eo.target_end = t1;
            if ((rc = run_walk(t, o.mlp_theta_est, eps, t->est_acc.p, nullptr, nullptr, nullptr, eo,
                               true)))
                return rc;
            rc = mlp_anorm(t, t->est_acc.p, nullptr, false);
        }
        if (rc) return rc;
        mac.kc = (const float *)t->kc.p;
        mac.anorm = (const float *)t->anorm.p;
        mac.tmax2 = (float)(o.mlp_theta_max * o.mlp_theta_max);
        mac.tau = (float)pow(10.0, o.mlp_log10_tau);
        dispatch2<float, true, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
    } else if (t->dtype == BH_F32) {
        if (o.order == 0) dispatch2<float, false, false>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        else dispatch2<float, true, false>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
    } else {
        if (o.order == 0) dispatch2<double, false, false>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        else dispatch2<double, true, false>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
    }
    return check_launch("walk");
}

}  // namespace bh
