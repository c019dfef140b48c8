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
#include <algorithm>
#include <type_traits>

#include "bh_internal.h"
#include "mlp.h"

namespace bh {
namespace {

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
// Square root for the acceptance tests: in FP32 the hardware's v_sqrt_f32
// (within 1 ulp) instead of the correctly rounded sequence sqrtf expands to
// (some fifteen instructions); the tests' decisions near a threshold are
// within the margin the oracle flags, far above an ulp.
__device__ __forceinline__ float tsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double tsqrt(double x) { return sqrt(x); }

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
    auto term = [&](const BodyRec<R> &s, int j) {
        // the lane's own body (SELF) contributes nothing: a select, not a
        // branch, so that the wave stays convergent
        const R dx = s.x - X, dy = s.y - Y, dz = s.z - Z;
        R r2 = dx * dx + eps2;
        r2 = dy * dy + r2;
        r2 = dz * dz + r2;
        R inv = rsq(r2);
        if (SELF) inv = j != i ? inv : (R)0;
        const R minv = s.m * inv;
        const R mi3 = minv * (inv * inv);
        px += mi3 * dx;
        py += mi3 * dy;
        pz += mi3 * dz;
        if (PHI) pq -= minv;
        if (CNT && SELF) cpp += j != i ? 1u : 0u;
    };
    int j = jb;
    for (; j + 4 <= je; j += 4) {  // four uniform loads in flight, then the terms in order
        const BodyRec<R> s0 = bodies[j], s1 = bodies[j + 1], s2 = bodies[j + 2],
                         s3 = bodies[j + 3];
        term(s0, j);
        term(s1, j + 1);
        term(s2, j + 2);
        term(s3, j + 3);
    }
    for (; j < je; ++j) term(bodies[j], j);
    if (CNT && !SELF) cpp += (uint32_t)(je - jb);
    sx += px;
    sy += py;
    sz += pz;
    if (PHI) sp += pq;
}

// Relative criteria of a walk (MAC: 0 opening angle, 1 error budget with
// k_C = 1, 2 / 3 the learned criterion with bf16 / fp16 network operands):
// per cell M l^3 (budget), per sorted rank |a_i|, the floor of |a_i|
// (device scalar), theta_max^2, tau, the packed network and the softening.
struct MlpMac {
    const float *kc;
    const float *anorm;
    const float *afloor;
    float tmax2, tau;
    const MlpPacked *net;
    float eps;
    const void *oct;  // order 3: octopole records, 8 values per node
    uint32_t *npq;    // optional: particle-cell terms with the quadrupole
};

// Criterion codes of the walk kernels: 0 opening angle, 1 error budget,
// 2 / 3 learned (bf16 / fp16 network), 4 error budget with the mixed order
// (per cell the monopole where its budget charged with the dropped
// quadrupole's bound holds, else the quadrupole, else open).
template <int MAC> constexpr bool kBudget = MAC == 1 || MAC == 4;
template <int MAC> constexpr bool kLearned = MAC == 2 || MAC == 3;

template <int MAC> struct NetVec { using type = bf16x8; };

// The error budget with monopole terms charges a cell the bound on the
// quadrupole term it drops (Sec. 2.2): |Q x / s^5 - (5/2) (x.Q.x) x / s^7|
// <= (7/2) |Q|_F / s^4, so the cell is accepted iff
// M l^3 + (7/2) |Q|_F d < tau |a| d^5.  This returns (7/2) |Q|_F of the
// record's traceless quadrupole.
template <typename Rec> __device__ __forceinline__ float quad_bound(const Rec &nd) {
    const float qxx = (float)nd.qxx, qyy = (float)nd.qyy, qzz = -qxx - qyy;
    const float qxy = (float)nd.qxy, qxz = (float)nd.qxz, qyz = (float)nd.qyz;
    const float diag = qxx * qxx + qyy * qyy + qzz * qzz;
    const float off = qxy * qxy + qxz * qxz + qyz * qyz;
    return 3.5f * tsqrt(2.f * off + diag);
}

// The octopole term of a particle-cell interaction (order 3; Sec. 2.2, the
// l = 3 term): from o = (xxx xxy xxz xyy xyz yyy yyz), the traceless
// octopole's independent components, and x = body - COM, adds
// (O:xx) / (2 s^7) - (7/6) (O:xxx) x / s^9 to the acceleration and
// -(O:xxx) / (6 s^7) to the potential; inv2 = 1/s^2, inv5 = 1/s^5.
template <typename R, bool PHI>
__device__ __forceinline__ void oct_term(const R *o, R x, R y, R z, R inv2, R inv5, R &sx,
                                         R &sy, R &sz, R &sp) {
    const R xzz = -o[0] - o[3], yzz = -o[1] - o[5], zzz = -o[2] - o[6];
    const R xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    const R vx = o[0] * xx + o[3] * yy + xzz * zz + (R)2 * (o[1] * xy + o[2] * xz + o[4] * yz);
    const R vy = o[1] * xx + o[5] * yy + yzz * zz + (R)2 * (o[3] * xy + o[4] * xz + o[6] * yz);
    const R vz = o[2] * xx + o[6] * yy + zzz * zz + (R)2 * (o[4] * xy + xzz * xz + yzz * yz);
    const R t3 = x * vx + y * vy + z * vz;
    const R inv7 = inv5 * inv2;
    const R c = (R)(7.0 / 6.0) * t3 * inv2;
    sx = inv7 * ((R)0.5 * vx - c * x) + sx;
    sy = inv7 * ((R)0.5 * vy - c * y) + sy;
    sz = inv7 * ((R)0.5 * vz - c * z) + sz;
    if (PHI) sp = sp - t3 * inv7 * (R)(1.0 / 6.0);
}
template <> struct NetVec<3> { using type = f16x8; };

__device__ __forceinline__ float lg10(float x) {
    return __builtin_amdgcn_logf(x) * 0.30102999566398120f;
}

// The per-body walk of one wavefront (see the file header): lane body i
// (live), its offset (ox, oy, oz) from its leaf centre (ax, ay, az), leaf
// index myleaf; sums into s*, counts into cpp/cpc.  With PF both possible
// successor records are loaded while a node is processed: this shortens the
// dependent chain of a lone wavefront (the group walk's per-body fallback)
// but costs the register file the occupancy that hides it in a full launch.
template <typename R, bool ORDER2, bool PHI, bool CNT, int MAC, bool PF = false,
          bool GUARD = false, bool OCT = false>
__device__ __forceinline__ void body_sweep(const typename NodeRecT<R>::type *__restrict__ nodes,
                                           int m, const BodyRec<R> *__restrict__ bodies,
                                           int nbodies, int i, bool live, R ox, R oy, R oz,
                                           R ax, R ay, R az, int myleaf, R theta2, R eps2,
                                           const MlpMac &mac, R &sx, R &sy, R &sz, R &sp,
                                           uint32_t &cpp, uint32_t &cpc, uint32_t &cpq) {
    using Rec = typename NodeRecT<R>::type;
    float tau_a = 0.f;  // tau |a_i|
    if (MAC >= 1 && live) tau_a = mac.tau * fmaxf(mac.anorm[i], *mac.afloor);
    const float lt = kLearned<MAC> && live ? lg10(tau_a) : 0.f;
    const int lane = (int)lane_id();

    const bool root_leaf = nodes[0].next == 1;
    int idx = root_leaf ? 0 : 1;
    int resume = live ? idx : 0x7fffffff;

    Rec nd_next = nodes[uniform(idx)];
    while (idx < m) {
        idx = uniform(idx);
        const Rec nd = PF ? nd_next : nodes[idx];
        const bool act = resume <= idx;
        const int nxt = uniform(nd.next);
        const int cnt = uniform(nd.count);
        Rec n1{}, n2{};
        if (PF) {
            const int s1 = uniform(idx + 1 < m ? idx + 1 : idx);
            const int s2 = uniform(nxt > idx && nxt < m ? nxt : s1);
            n1 = nodes[s1];
            n2 = nodes[s2];
        }
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
            bool mono = !ORDER2;  // the term without the quadrupole
            if (kBudget<MAC>) {
                // error budget: M l^3 / d^5 below tau |a_i|, l/d below
                // theta_max, and the body outside the cell
                // (monopole terms: plus the dropped quadrupole's bound)
                float kcv = mac.kc[idx];
                const R hs = (R)0.5 * tsqrt(nd.l2);
                const bool inside = fabs(X) <= hs && fabs(Y) <= hs && fabs(Z) <= hs;
                const R d = tsqrt(d2);
                const R rhs = tau_a * (d2 * d2 * d);
                const bool geo = act && nd.l2 < (R)mac.tmax2 * d2 && !inside;
                if (MAC == 4) {  // mixed: the monopole where it meets the budget
                    mono = geo && quad_bound(nd) * d + kcv < rhs;
                    accept = geo && kcv < rhs;
                } else {
                    if (!ORDER2) kcv = quad_bound(nd) * d + kcv;
                    accept = geo && kcv < rhs;
                }
            } else if (kLearned<MAC>) {
                // learned, the body as its own group: the network's error
                // for (body, cell) below tau |a_i|, l/d below theta_max, the
                // body outside the cell; one 64-row batch per node
                const R hs = (R)0.5 * tsqrt(nd.l2);
                const bool inside = fabs(X) <= hs && fabs(Y) <= hs && fabs(Z) <= hs;
                const bool cand = act && nd.l2 < (R)mac.tmax2 * d2 && !inside && nd.m > (R)0;
                accept = false;
                if (__ballot(cand)) {  // wave-uniform: the MFMAs need every lane
                    float f[kMlpIn] = {};
                    if (cand)
                        gfeatures<R>(-x, -y, -z, (R)0, (R)0, (R)0, nd.mx, nd.my, nd.mz, nd.m,
                                     nd.qxx, nd.qxy, nd.qxz, nd.qyy, nd.qyz, nd.l2, cnt,
                                     nxt == idx + 1, (R)mac.eps, f);
                    const float pred =
                        mlp_eval_p<typename NetVec<MAC>::type>(mac.net, f, lane);
                    accept = cand && pred + lg10((float)nd.m) + 1.5f * lg10((float)nd.l2) -
                                             2.5f * lg10((float)d2) < lt;
                }
            } else {
                accept = act && nd.l2 < theta2 * d2;
                // containment guard: a cell holding the body is opened.  Below
                // theta^2 = 1/3 no such cell passes the test (d is at most the
                // cube's diagonal); the margin covers the rounding of d2.
                if (GUARD && theta2 > (R)0.33) {
                    const R q = (R)0.25 * nd.l2;  // (side / 2)^2, exact
                    accept = accept && !(X * X <= q && Y * Y <= q && Z * Z <= q);
                }
            }
            if (accept) {  // skipped as a whole when no lane accepts
                const R inv = rsq(d2 + eps2);
                const R inv2 = inv * inv;
                const R inv3 = inv * inv2;
                if (ORDER2) {
                    // (mixed order: a monopole lane takes Q = 0, which gives
                    // the monopole term exactly)
                    const R qs = MAC == 4 && mono ? (R)0 : (R)1;
                    const R qxx = nd.qxx * qs, qxy = nd.qxy * qs, qxz = nd.qxz * qs,
                            qyy = nd.qyy * qs, qyz = nd.qyz * qs;
                    const R qzz = -qxx - qyy;
                    const R qx = qxx * x + qxy * y + qxz * z;
                    const R qy = qxy * x + qyy * y + qyz * z;
                    const R qz = qxz * x + qyz * y + qzz * z;
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
                    if (OCT)
                        oct_term<R, PHI>((const R *)mac.oct + 8 * (int64_t)idx, x, y, z, inv2,
                                         inv5, sx, sy, sz, sp);
                } else {
                    const R g = nd.m * inv3;
                    sx = -g * x + sx;
                    sy = -g * y + sy;
                    sz = -g * z + sz;
                    if (PHI) sp = sp - nd.m * inv;
                }
                if (CNT) {
                    ++cpc;
                    if (!mono) ++cpq;
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
        const int nidx = any_open ? idx + 1 : (nxt > idx ? nxt : idx + 1);  // always moves forward
        if (PF) nd_next = nidx == idx + 1 ? n1 : n2;
        idx = nidx;
    }
}

template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED_OUT, int MAC,
          bool GUARD, bool OCT>
__global__ __launch_bounds__(256) void k_walk(
    const typename NodeRecT<R>::type *__restrict__ nodes, int m,
    const BodyRec<R> *__restrict__ bodies, const Anchor<R> *__restrict__ anchors,
    const uint32_t *__restrict__ perm, int nbodies, int t0, int t1, int nwaves_padded,
    R theta2, R eps2, R *__restrict__ acc, R *__restrict__ phi_out,
    uint32_t *__restrict__ npp_out, uint32_t *__restrict__ npc_out, MlpMac mac) {
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
    uint32_t cpp = 0, cpc = 0, cpq = 0;
    body_sweep<R, ORDER2, PHI, CNT, MAC, false, GUARD, OCT>(nodes, m, bodies, nbodies, i, live, ox,
                                                       oy, oz, ax, ay, az, myleaf, theta2, eps2,
                                                       mac, sx, sy, sz, sp, cpp, cpc, cpq);
    if (live) {
        const int o = SORTED_OUT ? i : (int)perm[i];
        acc[3 * (int64_t)o + 0] = sx;
        acc[3 * (int64_t)o + 1] = sy;
        acc[3 * (int64_t)o + 2] = sz;
        if (PHI) phi_out[o] = sp;
        if (CNT) {
            npp_out[o] = cpp;
            npc_out[o] = cpc;
            if (mac.npq) mac.npq[o] = cpq;
        }
    }
}

template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED, int MAC, bool GUARD,
          bool OCT>
void launch(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
            uint32_t *npp, uint32_t *npc, const MlpMac &mac) {
    const int nw = div_up(t1 - t0, 64);
    const int nblk = div_up(nw, 4);
    const int nblk_pad = div_up(nblk, 64) * 64;
    if (t->ctx->walk_ev) hipEventRecord(t->ctx->walk_ev[0], t->ctx->stream);
    k_walk<R, ORDER2, PHI, CNT, SORTED, MAC, GUARD, OCT><<<nblk_pad, 256, 0, t->ctx->stream>>>(
        (const typename NodeRecT<R>::type *)t->recs.p, (int)t->m,
        (const BodyRec<R> *)t->bodies.p, (const Anchor<R> *)t->anchors.p, t->perm, (int)t->n, t0,
        t1, nblk_pad * 4, (R)(theta * theta), (R)(eps * eps), (R *)acc, (R *)phi, npp, npc, mac);
    if (t->ctx->walk_ev) hipEventRecord(t->ctx->walk_ev[1], t->ctx->stream);
}

template <typename R, bool ORDER2, int MAC, bool GUARD = false, bool OCT = false>
void dispatch2(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
               uint32_t *npp, uint32_t *npc, bool sorted, const MlpMac &mac) {
    const bool P = phi != nullptr, C = npp != nullptr;
#define BH_W(p, c, s) launch<R, ORDER2, p, c, s, MAC, GUARD, OCT>(t, t0, t1, theta, eps, acc, phi, npp, npc, mac)
    if (sorted) {  // simulation walks: phi for the energy, counts when recorded
        if (P) BH_W(true, false, true);
        else if (C) BH_W(false, true, true);
        else BH_W(false, false, true);
    } else if (P && C) BH_W(true, true, false);
    else if (P) BH_W(true, false, false);
    else if (C) BH_W(false, true, false);
    else BH_W(false, false, false);
#undef BH_W
}


// ---------------------------------------------------------------- group walk
// One wavefront = one group of 64 consecutive sorted bodies, one decision
// per cell for the whole group: the cell is accepted iff its cube does not
// meet the group's bounding box and side < theta * d_g (opening angle) or,
// error budget, side < theta_max * d_g and k_C M l^3 < tau a_min d_g^5,
// with d_g the distance from the cell's COM to the box and a_min the
// smallest |a_i| of the group.  Since every decision is wave-uniform, no lane
// idles while others descend, and the tests themselves run lane-parallel:
// the wave pops up to 64 nodes from a stack in LDS, each lane classifies
// one, children of opened nodes are pushed (child table, prefix sum over
// the lanes), then every lane evaluates each accepted cell and each
// particle-particle leaf of the round with its own body.  If the children
// would overflow the stack, the opened subtrees are walked one at a time
// by a sequential pre-order sweep that needs no memory.
//
// A group spread over a large region (64 bodies consecutive on the
// space-filling curve can straddle one of its jumps) would open nearly
// everything.  The group's work (particle-cell terms plus particle-particle
// bodies, the same for each of its bodies) is therefore capped: a group
// that would exceed the cap drops its partial sums and is walked per body
// with the same criterion instead.
constexpr int kGroupStack = 640;       // LDS stack entries per wavefront
constexpr int kStageW = 12;            // LDS words per staged accepted cell
// bodies of particle-particle leaves staged per batch (4 words each, in the
// same LDS as the accepted cells)
// with the octopole (order 3) a staged cell also carries its 7 components
template <bool OCT> struct StageW { static constexpr int value = OCT ? 20 : kStageW; };
// Default per-group work caps: a fallback walks the group per body at a
// quarter of the lanes, so the cap sits near three times a typical group's
// work (about 1300 per body for the error budget, 1600-2200 for the learned
// and opening-angle criteria at rms 1e-3).
constexpr int kGroupWorkCap = 6144;        // opening angle, learned criterion
constexpr int kGroupWorkCapBudget = 4096;  // error budget with k_C = 1

struct GroupMac {
    const float *kc;     // error budget: M l^3 per node (k_C = 1)
    const float *anorm;  // |a_i| per sorted rank
    const float *afloor;  // floor of |a_i| (device scalar)
    float tau;
    int cap;             // stack entries used (<= kGroupStack)
    int work_cap;        // per-group work above which the group walks per body
    // work items in hand-out order, per XCD chunk of groups (chunk c's at
    // kParts * its first group): 16 g + 15 walks group g, 16 g + q
    // (q < kParts) walks lanes kPartLanes q .. kPartLanes (q + 1) - 1 of
    // group g per body; or null: groups in index order
    const uint32_t *items;
    // per group: further walks for which the group is predicted to exceed
    // the work cap (written when a one-run group does), then (at ng + g)
    // the length of its last prediction; or null
    uint8_t *gfb;
    int predict_first;   // walks predicted after a first excess
    const MlpPacked *net;  // learned criterion: the packed network
    float eps;             // and the softening (a feature)
    const void *oct;       // order 3: octopole records, 8 values per node
    uint32_t *npq;         // optional: particle-cell terms with the quadrupole
};

// A group that exceeded the work cap is walked per body straight away (in
// parts of kPartLanes bodies, separate items) in the next walks, then the
// group walk is tried again.  An excess found during a walk is paid on the
// wavefront that found it (the group walk up to the cap, then the per-body
// walk), late in the launch; a wrong prediction costs the per-body walk of
// a group that would fit.  With few groups per resident wavefront the late
// excess is a tail on a short launch: the prediction then lasts
// kPredictWalks walks.  With many, the tail is spread thin, and in a
// simulation the groups over the cap may turn over within a step or two
// (bodies near heavy ones): the prediction then lasts one walk after a first
// excess and doubles with each excess that follows an expired one, up to
// kPredictWalks.  A group walk that fits resets it.
constexpr int kPredictWalks = 15;
constexpr int kLongPredictGroupsPerWave = 4;
constexpr int kPartLanes = 16;
constexpr int kParts = 64 / kPartLanes;
constexpr uint32_t kWholeGroup = 15;

template <typename R>
__device__ __forceinline__ R wave_min(R v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) v = fmin(v, __shfl_xor(v, s));
    return v;
}
template <typename R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) v = fmax(v, __shfl_xor(v, s));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) v = min(v, __shfl_xor(v, sh));
    return __builtin_amdgcn_readfirstlane(v);
}

// kGCand: a candidate of the learned criterion, decided by the network
// kGPQ: accepted with the quadrupole (the mixed order; kGPC is then the
// monopole)
enum : int { kGNone = 0, kGPC = 1, kGPP = 2, kGOpen = 3, kGCand = 4, kGPQ = 5 };

// One group: the 64 bodies of sorted rank [base, min(base + 64, t1)).
template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED_OUT, int MAC, bool OCT>
__device__ __forceinline__ auto group_walk(
    const typename NodeRecT<R>::type *__restrict__ nodes, int m,
    const BodyRec<R> *__restrict__ bodies, const Anchor<R> *__restrict__ anchors,
    const int4 *__restrict__ kids, const uint32_t *__restrict__ perm, int nbodies, int base,
    int t1, R theta2, R eps2, R *__restrict__ acc, R *__restrict__ phi_out,
    uint32_t *__restrict__ npp_out, uint32_t *__restrict__ npc_out, const GroupMac &gm,
    int *__restrict__ stk, R *__restrict__ stage, const int8_t *__restrict__ delta,
    const int32_t *__restrict__ level) -> bool {
    using Rec = typename NodeRecT<R>::type;
    constexpr int SW = StageW<OCT>::value;    // LDS words per staged cell
    constexpr int PPS = 64 * SW / 4;          // bodies per particle-particle batch
    const int lane = (int)lane_id();
    const int i = base + lane;
    const bool live = i < t1;
    const int g_end = min(base + 64, t1);
    int runs = 0, over = 0;  // runs walked, runs over the work cap

    R ox = 0, oy = 0, oz = 0, ax = 0, ay = 0, az = 0;
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
    // A group that straddles a jump of the space-filling curve is split into
    // runs of consecutive bodies, each walked as a group of its own: from
    // the left, a run [lo, hi) is cut at its first largest jump (the first
    // smallest common-prefix length of adjacent keys) while its common cell
    // lies more than two levels above its shallowest leaf.
    const int dl = (live && lane > 0) ? (int)delta[i] : 127;  // common octal digits with i - 1
    const int lv = live ? level[myleaf] : 127;
    const int nlive = g_end - base;

    auto pass = [&](const int lo, const int hi) {
        const bool live_run = live && lane >= lo && lane < hi;
        // the group's bounding box, relative to the leaf centre g of the first
        // body: grid centres differ exactly, so the box and the cell distances
        // are accurate to the rounding of the offsets
        const R gx = __shfl(ax, lo), gy = __shfl(ay, lo), gz = __shfl(az, lo);
        const R big = (R)3.0e38;
        const R px = (ax - gx) + ox, py = (ay - gy) + oy, pz = (az - gz) + oz;
        const R lx = wave_min(live_run ? px : big), ly = wave_min(live_run ? py : big),
                lz = wave_min(live_run ? pz : big);
        const R hx = wave_max(live_run ? px : -big), hy = wave_max(live_run ? py : -big),
                hz = wave_max(live_run ? pz : -big);
        const R bcx = (R)0.5 * (lx + hx), bcy = (R)0.5 * (ly + hy), bcz = (R)0.5 * (lz + hz);
        const R bhx = (R)0.5 * (hx - lx), bhy = (R)0.5 * (hy - ly), bhz = (R)0.5 * (hz - lz);
        float tau_amin = 0.f;
        if (MAC >= 1)
            tau_amin = gm.tau * fmaxf(wave_min(live_run ? gm.anorm[i] : 3.0e38f), *gm.afloor);
        const float lt = kLearned<MAC> ? lg10(tau_amin) : 0.f;  // log10(tau a_min)

        R sx = 0, sy = 0, sz = 0, sp = 0;
        uint32_t cpp = 0, cpc = 0, cpq = 0;
        int work = 0;  // wave-uniform

        // decision for node c (any lane; wave-uniform when the node is)
        auto classify = [&](const Rec &nd, int c, float kcv) -> int {
            if (c == 0) return kGOpen;  // the root is always opened
            if (nd.count == 1) return kGPP;
            const R hs = (R)0.5 * tsqrt(nd.l2);
            const R ux = (nd.cx - gx) - bcx, uy = (nd.cy - gy) - bcy, uz = (nd.cz - gz) - bcz;
            const bool overlap = fabs(ux) <= hs + bhx && fabs(uy) <= hs + bhy && fabs(uz) <= hs + bhz;
            const R tx = fmax(fabs(ux + nd.mx) - bhx, (R)0);
            const R ty = fmax(fabs(uy + nd.my) - bhy, (R)0);
            const R tz = fmax(fabs(uz + nd.mz) - bhz, (R)0);
            const R dg2 = tx * tx + ty * ty + tz * tz;
            bool accept = !overlap && nd.l2 < theta2 * dg2;
            if (kBudget<MAC>) {  // (monopole terms: plus the dropped quadrupole's bound)
                const float dg = tsqrt((float)dg2);
                const float rhs = tau_amin * (float)(dg2 * dg2 * dg);
                if (MAC == 4) {  // mixed order: the monopole where it meets the budget
                    if (accept && quad_bound(nd) * dg + kcv < rhs) return kGPC;
                    if (accept && kcv < rhs) return kGPQ;
                    accept = false;
                } else {
                    if (!ORDER2) kcv = quad_bound(nd) * dg + kcv;
                    accept = accept && kcv < rhs;
                }
            }
            if (kLearned<MAC> && accept && nd.m > (R)0) return kGCand;  // the network decides
            if (kLearned<MAC>) accept = false;
            if (accept) return MAC == 4 ? kGPQ : kGPC;
            return nd.next == c + 1 ? kGPP : kGOpen;
        };
        // the learned decision for the candidates among the lanes' nodes:
        // every lane calls (the MFMAs need the whole wave); cls is updated
        // on the candidate lanes
        auto learn = [&](const Rec &nd, int c, int &cls) {
            float f[kMlpIn] = {};
            R dg2 = (R)1;
            if (cls == kGCand) {
                const R ux = ((nd.cx - gx) - bcx) + nd.mx, uy = ((nd.cy - gy) - bcy) + nd.my,
                        uz = ((nd.cz - gz) - bcz) + nd.mz;
                dg2 = gfeatures<R>(ux, uy, uz, bhx, bhy, bhz, nd.mx, nd.my, nd.mz, nd.m, nd.qxx,
                                   nd.qxy, nd.qxz, nd.qyy, nd.qyz, nd.l2, nd.count,
                                   nd.next == c + 1, (R)gm.eps, f);
            }
            const float pred = mlp_eval_p<typename NetVec<MAC>::type>(gm.net, f, lane);
            if (cls == kGCand)
                cls = pred + lg10((float)nd.m) + 1.5f * lg10((float)nd.l2) -
                                  2.5f * lg10((float)dg2) < lt
                          ? kGPC
                          : (nd.next == c + 1 ? kGPP : kGOpen);
        };
        // particle-cell term of node nd for this lane's body
        // (quad: with the quadrupole, in a walk of order 2 or more)
        auto cell_term = [&](const Rec &nd, int c, bool quad) {
            const R X = (ax - nd.cx) + ox, Y = (ay - nd.cy) + oy, Z = (az - nd.cz) + oz;
            const R x = X - nd.mx, y = Y - nd.my, z = Z - nd.mz;
            const R d2 = x * x + y * y + z * z;
            const R inv = rsq(d2 + eps2);
            const R inv2 = inv * inv;
            const R inv3 = inv * inv2;
            if (ORDER2 && quad) {
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
                if (OCT)
                    oct_term<R, PHI>((const R *)gm.oct + 8 * (int64_t)c, x, y, z, inv2, inv5, sx,
                                     sy, sz, sp);
            } else {
                const R g = nd.m * inv3;
                sx = -g * x + sx;
                sy = -g * y + sy;
                sz = -g * z + sz;
                if (PHI) sp = sp - nd.m * inv;
            }
            if (CNT) {
                ++cpc;
                if (ORDER2 && quad) ++cpq;
            }
            ++work;
        };
        // particle-cell term of a staged cell: COM relative to the group origin
        // g, mass, quadrupole (xx xy xz yy yz zz)
        // (Quad: an integral constant, with the quadrupole)
        auto staged_term = [&](const R *st, auto Quad) {
            const R x = px - st[0], y = py - st[1], z = pz - st[2];
            const R s2 = z * z + (y * y + (x * x + eps2));
            const R inv = rsq(s2);
            const R inv2 = inv * inv;
            const R m = st[3];
            if constexpr (decltype(Quad)::value) {
                // a = inv^5 (Q x - (m s^2 + 5/2 (x.Q.x)/s^2) x)
                const R qx = st[4] * x + st[5] * y + st[6] * z;
                const R qy = st[5] * x + st[7] * y + st[8] * z;
                const R qz = st[6] * x + st[8] * y + st[9] * z;
                const R xqx = x * qx + y * qy + z * qz;
                const R inv5 = inv * (inv2 * inv2);
                const R c = m * s2 + ((R)2.5 * inv2) * xqx;
                sx = inv5 * (qx - c * x) + sx;
                sy = inv5 * (qy - c * y) + sy;
                sz = inv5 * (qz - c * z) + sz;
                if (PHI) sp = sp - m * inv - (R)0.5 * (xqx * inv5);
                if (OCT) oct_term<R, PHI>(st + 10, x, y, z, inv2, inv5, sx, sy, sz, sp);
            } else {
                const R inv3 = inv * inv2;
                const R g = m * inv3;
                sx = -g * x + sx;
                sy = -g * y + sy;
                sz = -g * z + sz;
                if (PHI) sp = sp - m * inv;
            }
            if (CNT) {
                ++cpc;
                if (decltype(Quad)::value) ++cpq;
            }
        };
        // particle-particle terms with the bodies of leaf (or one-body cell) nd
        auto leaf_terms = [&](const Rec &nd) {
            const int jb = uniform(nd.begin);
            const int je = min(jb + uniform(nd.count), nbodies);  // guard
            const R X = (ax - nd.cx) + ox, Y = (ay - nd.cy) + oy, Z = (az - nd.cz) + oz;
            work += je - jb;
            if (jb < g_end && je > base)  // holds bodies of the group: skip self
                leaf_pp<R, PHI, CNT, true>(bodies, jb, je, i, X, Y, Z, eps2, sx, sy, sz, sp, cpp);
            else
                leaf_pp<R, PHI, CNT, false>(bodies, jb, je, i, X, Y, Z, eps2, sx, sy, sz, sp, cpp);
        };
        // the subtree below node r without the stack (overflow path)
        auto sweep = [&](int r0) {
            int idx = uniform(r0) + 1;
            const int end = uniform(nodes[uniform(r0)].next);
            while (idx < end && work <= gm.work_cap) {
                idx = uniform(idx);
                const Rec nd = nodes[idx];
                int cls = uniform(classify(nd, idx, kBudget<MAC> ? gm.kc[idx] : 0.f));
                if (kLearned<MAC> && cls == kGCand) {
                    learn(nd, idx, cls);
                    cls = uniform(cls);
                }
                if (cls == kGPC) cell_term(nd, idx, ORDER2 && MAC != 4);
                else if (cls == kGPQ) cell_term(nd, idx, true);
                else if (cls == kGPP) leaf_terms(nd);
                const int nx = uniform(nd.next);
                idx = cls == kGOpen || nx <= idx ? idx + 1 : nx;  // always moves forward
            }
        };

        if (nodes[0].next == 1) {  // the root is a leaf
            leaf_terms(nodes[0]);
        } else {
            if (lane == 0) stk[0] = 0;
            int top = 1;  // wave-uniform stack size
            while (top > 0 && work <= gm.work_cap) {
                top = uniform(top);
                const int k = min(top, 64);
                top -= k;
                __builtin_amdgcn_wave_barrier();
                const bool has = lane < k;
                // lanes without a node load and classify the root (valid,
                // cached) and take no part
                const int c = has ? stk[top + lane] : 0;
                int4 k0 = make_int4(-1, -1, -1, -1), k1 = k0;
                if (!kLearned<MAC>) {
                    k0 = kids[2 * (int64_t)c];  // loaded with the record, used if opened
                    k1 = kids[2 * (int64_t)c + 1];
                }
                const Rec nd = nodes[c];
                int cls = classify(nd, c, kBudget<MAC> ? gm.kc[c] : 0.f);
                if (!has) cls = kGNone;
                if (kLearned<MAC>) {
                    // the children after the network (fewer registers live
                    // across its evaluation)
                    if (__ballot(cls == kGCand)) learn(nd, c, cls);
                    if (cls == kGOpen) {
                        k0 = kids[2 * (int64_t)c];
                        k1 = kids[2 * (int64_t)c + 1];
                    }
                }
                const uint64_t m_pc = __ballot(cls == kGPC);  // (mixed order: monopoles)
                const uint64_t m_pq = MAC == 4 ? __ballot(cls == kGPQ) : 0ull;
                const uint64_t m_pp = __ballot(cls == kGPP);
                const uint64_t m_op = __ballot(cls == kGOpen);
                // stage the accepted cell for every lane; in the mixed order
                // the quadrupole terms from slot 0 up, the monopoles from slot
                // 63 down (at most 64 cells a round)
                const bool quad_st = MAC == 4 ? cls == kGPQ : ORDER2;
                if (cls == kGPC || (MAC == 4 && cls == kGPQ)) {
                    const uint64_t mm = MAC == 4 && cls == kGPQ ? m_pq : m_pc;
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                    R *st = stage + SW * (MAC == 4 && cls == kGPC ? 63 - rank : rank);
                    st[0] = (nd.cx - gx) + nd.mx;
                    st[1] = (nd.cy - gy) + nd.my;
                    st[2] = (nd.cz - gz) + nd.mz;
                    st[3] = nd.m;
                    if (ORDER2 && quad_st) {
                        st[4] = nd.qxx;
                        st[5] = nd.qxy;
                        st[6] = nd.qxz;
                        st[7] = nd.qyy;
                        st[8] = nd.qyz;
                        st[9] = -nd.qxx - nd.qyy;
                    }
                    if (OCT) {
                        const R *o = (const R *)gm.oct + 8 * (int64_t)c;
                        for (int q = 0; q < 7; ++q) st[10 + q] = o[q];
                    }
                }
                if (m_op) {
                    const int kid[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
                    // the child table lists a cell's children first (then -1):
                    // their count by bisection
                    int nk = 0;
                    if (cls == kGOpen) {
                        if (k0.w >= 0)
                            nk = k1.y >= 0 ? (k1.w >= 0 ? 8 : k1.z >= 0 ? 7 : 6)
                                           : (k1.x >= 0 ? 5 : 4);
                        else
                            nk = k0.y >= 0 ? (k0.z >= 0 ? 3 : 2) : (k0.x >= 0 ? 1 : 0);
                    }
                    // exclusive prefix sum of nk (0..8) over the lanes, bit by bit
                    int excl = 0, total = 0;
    #pragma unroll
                    for (int bit = 0; bit < 4; ++bit) {
                        const uint64_t bm = __ballot((nk >> bit) & 1);
                        excl += (int)__builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))
                                << bit;
                        total += __builtin_popcountll(bm) << bit;
                    }
                    if (top + total <= gm.cap) {
                        const int off = top + excl;
#pragma unroll
                        for (int q = 0; q < 8; ++q)  // constant offsets, no indexed registers
                            if (q < nk) stk[off + q] = kid[q];
                        top += total;
                    } else {
                        uint64_t mm = m_op;
                        while (mm) {
                            const int bit = __builtin_ctzll(mm);
                            mm &= mm - 1;
                            sweep(__builtin_amdgcn_readlane(c, bit));
                        }
                    }
                }
                // accepted cells from LDS (same address on every lane: broadcast)
                const int npc_round = __builtin_popcountll(m_pc);
                const int npq_round = MAC == 4 ? __builtin_popcountll(m_pq) : 0;
                __builtin_amdgcn_wave_barrier();
                // two cells per iteration (immediate LDS offsets, two
                // independent chains; the sums still follow q)
                using QuadT = std::integral_constant<bool, ORDER2 && MAC != 4>;
                if (MAC == 4) {
                    const std::true_type yes;
                    int q = 0;
                    for (; q + 1 < npq_round; q += 2) {
                        staged_term(stage + SW * q, yes);
                        staged_term(stage + SW * (q + 1), yes);
                    }
                    if (q < npq_round) staged_term(stage + SW * q, yes);
                }
                {
                    const QuadT quad;
                    const int top_slot = MAC == 4 ? 63 : 0, dir = MAC == 4 ? -1 : 1;
                    int q = 0;
                    for (; q + 1 < npc_round; q += 2) {
                        staged_term(stage + SW * (top_slot + dir * q), quad);
                        staged_term(stage + SW * (top_slot + dir * (q + 1)), quad);
                    }
                    if (q < npc_round) staged_term(stage + SW * (top_slot + dir * q), quad);
                }
                work += npc_round + npq_round;
                // particle-particle leaves (and one-body cells) of the round.
                // The bodies of those that hold none of the group's bodies are
                // written to LDS in the group's frame, each leaf by its own
                // lane, as many as fit, and summed in one loop with no per-leaf
                // set-up; a leaf holding group bodies (the self term) or too
                // large to fit alone takes leaf_terms.
                int jb_l = 0, nb_l = 0;
                bool self_l = false;
                if (cls == kGPP) {
                    jb_l = nd.begin;
                    nb_l = max(0, min(nd.count, nbodies - jb_l));  // guard
                    self_l = jb_l < g_end && jb_l + nb_l > base;
                }
                const uint64_t m_self = __ballot(cls == kGPP && self_l);
                uint64_t pend = m_pp & ~m_self;
                while (pend) {
                    const bool mine = (pend >> lane) & 1;
                    const int nb = mine ? nb_l : 0;
                    int incl = nb;  // inclusive prefix sum over the lanes
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int v = __shfl_up(incl, o);
                        if (lane >= o) incl += v;
                    }
                    const bool fits = mine && incl <= PPS;
                    const uint64_t put = __ballot(fits);
                    if (put == 0) {  // the first pending leaf alone does not fit
                        const int bit = __builtin_ctzll(pend);
                        pend &= pend - 1;
                        leaf_terms(nodes[__builtin_amdgcn_readlane(c, bit)]);
                        continue;
                    }
                    pend &= ~put;
                    __builtin_amdgcn_wave_barrier();
                    if (fits) {
                        const R lx = nd.cx - gx, ly = nd.cy - gy, lz = nd.cz - gz;  // exact
                        R *d = stage + 4 * (incl - nb);
                        const BodyRec<R> *src = bodies + jb_l;
                        auto put_body = [&](int q, const BodyRec<R> &sb) {
                            d[4 * q + 0] = lx + sb.x;
                            d[4 * q + 1] = ly + sb.y;
                            d[4 * q + 2] = lz + sb.z;
                            d[4 * q + 3] = sb.m;
                        };
                        int q = 0;
                        for (; q + 4 <= nb; q += 4) {  // four loads in flight
                            const BodyRec<R> b0 = src[q], b1 = src[q + 1], b2 = src[q + 2],
                                             b3 = src[q + 3];
                            put_body(q, b0);
                            put_body(q + 1, b1);
                            put_body(q + 2, b2);
                            put_body(q + 3, b3);
                        }
                        for (; q < nb; ++q) put_body(q, src[q]);
                    }
                    const int total =
                        __builtin_amdgcn_readlane(incl, 63 - __builtin_clzll(put));
                    __builtin_amdgcn_wave_barrier();
                    work += total;
                    if (CNT) cpp += (uint32_t)total;
                    // same address on every lane; two bodies per iteration
                    // (immediate LDS offsets, two independent chains; the
                    // sums still follow q)
                    auto pp_term = [&](const R *sb) {
                        const R dx = sb[0] - px, dy = sb[1] - py, dz = sb[2] - pz;
                        R r2 = dx * dx + eps2;
                        r2 = dy * dy + r2;
                        r2 = dz * dz + r2;
                        const R inv = rsq(r2);
                        const R minv = sb[3] * inv;
                        const R mi3 = minv * (inv * inv);
                        sx = mi3 * dx + sx;
                        sy = mi3 * dy + sy;
                        sz = mi3 * dz + sz;
                        if (PHI) sp = sp - minv;
                    };
                    int q = 0;
                    for (; q + 1 < total; q += 2) {
                        pp_term(stage + 4 * q);
                        pp_term(stage + 4 * (q + 1));
                    }
                    if (q < total) pp_term(stage + 4 * q);
                    __builtin_amdgcn_wave_barrier();
                }
                uint64_t mm = m_self;
                while (mm) {
                    const int bit = __builtin_ctzll(mm);
                    mm &= mm - 1;
                    leaf_terms(nodes[__builtin_amdgcn_readlane(c, bit)]);
                }
            }
        }
        const bool per_body = work > gm.work_cap;
        ++runs;
        over += per_body ? 1 : 0;
        if (per_body) {  // too spread out for one decision: walk per body
            sx = sy = sz = sp = 0;
            cpp = cpc = cpq = 0;
            const MlpMac pm{gm.kc, gm.anorm, gm.afloor, (float)theta2, gm.tau, gm.net, gm.eps, gm.oct, nullptr};
            body_sweep<R, ORDER2, PHI, CNT, MAC, !kLearned<MAC>, false, OCT>(nodes, m, bodies, nbodies, i, live_run, ox, oy, oz,
                                                    ax, ay, az, myleaf, theta2, eps2, pm, sx, sy, sz,
                                                    sp, cpp, cpc, cpq);
        }
        if (live_run) {
            const int o = SORTED_OUT ? i : (int)perm[i];
            acc[3 * (int64_t)o + 0] = sx;
            acc[3 * (int64_t)o + 1] = sy;
            acc[3 * (int64_t)o + 2] = sz;
            if (PHI) phi_out[o] = sp;
            if (CNT) {
                npp_out[o] = cpp;
                npc_out[o] = cpc;
                if (gm.npq) gm.npq[o] = cpq;
            }
        }
    };

    int lo = 0;
    while (lo < nlive) {
        int hi = nlive;
        while (hi - lo >= 2) {
            const int kanc = wave_min_i(lane > lo && lane < hi ? dl : 127);
            const int kleaf = wave_min_i(lane >= lo && lane < hi ? lv : 127);
            if (kanc >= kleaf - 2) break;
            const uint64_t at = __ballot(lane > lo && lane < hi && dl == kanc);
            hi = __builtin_ctzll(at);
        }
        pass(lo, hi);
        lo = hi;
    }
    return runs == 1 && over == 1;  // one run, walked per body
}

// Per-body walk of lanes q0 .. q0 + kPartLanes - 1 of the group at rank
// base (one part of a group predicted to exceed the work cap); the other
// lanes idle.  Each body's walk is the per-body walk's, whichever bodies share
// the wavefront.
template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED_OUT, int MAC, bool OCT>
__device__ __forceinline__ void part_walk(
    const typename NodeRecT<R>::type *__restrict__ nodes, int m,
    const BodyRec<R> *__restrict__ bodies, const Anchor<R> *__restrict__ anchors,
    const uint32_t *__restrict__ perm, int nbodies, int base, int q0, int t1, R theta2, R eps2,
    R *__restrict__ acc, R *__restrict__ phi_out, uint32_t *__restrict__ npp_out,
    uint32_t *__restrict__ npc_out, const GroupMac &gm) {
    const int lane = (int)lane_id();
    const bool live = lane < kPartLanes && base + q0 + lane < t1;
    const int i = live ? base + q0 + lane : base;  // idle lanes: any rank of the group
    R ox = 0, oy = 0, oz = 0, ax = 0, ay = 0, az = 0;
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
    uint32_t cpp = 0, cpc = 0, cpq = 0;
    const MlpMac pm{gm.kc, gm.anorm, gm.afloor, (float)theta2, gm.tau, gm.net, gm.eps, gm.oct, nullptr};
    body_sweep<R, ORDER2, PHI, CNT, MAC, !kLearned<MAC>, false, OCT>(nodes, m, bodies, nbodies, i, live, ox, oy, oz,
                                                  ax, ay, az, myleaf, theta2, eps2, pm, sx, sy, sz,
                                                  sp, cpp, cpc, cpq);
    if (live) {
        const int o = SORTED_OUT ? i : (int)perm[i];
        acc[3 * (int64_t)o + 0] = sx;
        acc[3 * (int64_t)o + 1] = sy;
        acc[3 * (int64_t)o + 2] = sz;
        if (PHI) phi_out[o] = sp;
        if (CNT) {
            npp_out[o] = cpp;
            npc_out[o] = cpc;
            if (gm.npq) gm.npq[o] = cpq;
        }
    }
}

// Groups are handed out dynamically: the groups are split into 8
// contiguous chunks, one per XCD (workgroups are dispatched to the XCDs in
// turn, so blockIdx % 8 names the XCD and a chunk's nodes stay in one L2),
// and every resident wavefront takes the next group of its chunk from an
// atomic counter until the chunk is done.  A heavy group then delays only
// the wavefront that drew it.
template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED_OUT, int MAC, bool OCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kLearned<MAC> ? 4 : 1))) void k_gwalk(
    const typename NodeRecT<R>::type *__restrict__ nodes, int m,
    const BodyRec<R> *__restrict__ bodies, const Anchor<R> *__restrict__ anchors,
    const int4 *__restrict__ kids, const uint32_t *__restrict__ perm, int nbodies, int t0,
    int t1, uint32_t *__restrict__ queue, R theta2, R eps2, R *__restrict__ acc,
    R *__restrict__ phi_out, uint32_t *__restrict__ npp_out, uint32_t *__restrict__ npc_out,
    GroupMac gm, const int8_t *__restrict__ delta, const int32_t *__restrict__ level) {
    __shared__ int stack_all[4][kGroupStack];
    __shared__ R stage_all[4][64 * StageW<OCT>::value];
    // the learned criterion's network, staged once per workgroup
    __shared__ u32x4 net_lds[kLearned<MAC> ? sizeof(MlpPacked) / 16 : 1];
    int *stk = stack_all[threadIdx.x >> 6];
    R *stage = stage_all[threadIdx.x >> 6];
    if (kLearned<MAC>) {
        const u32x4 *src = (const u32x4 *)gm.net;
        for (int k = threadIdx.x; k < (int)(sizeof(MlpPacked) / 16); k += 256) net_lds[k] = src[k];
        __syncthreads();
        gm.net = (const MlpPacked *)net_lds;
    }
    const int ng = (t1 - t0 + 63) / 64;
    const int xcd = (int)(blockIdx.x & 7);
    const int chunk = (ng + 7) / 8;
    const int g_lo = xcd * chunk, g_hi = min(ng, g_lo + chunk);
    uint32_t *ctr = queue + 64 * xcd;  // one counter per 256 bytes
    // item count of the chunk (written by the ordering kernel), or groups
    const int n_items = gm.items ? (int)queue[64 * xcd + 16] : g_hi - g_lo;
    for (;;) {
        uint32_t slot = 0;
        if (lane_id() == 0) slot = atomicAdd(ctr, 1u);
        const int gi = (int)__builtin_amdgcn_readfirstlane(slot);
        if (gi >= n_items) break;
        int g = g_lo + gi, code = (int)kWholeGroup;
        if (gm.items) {
            const uint32_t it = gm.items[kParts * (size_t)g_lo + gi];
            g = (int)(it >> 4);
            code = (int)(it & 15u);
        }
        if (code < kParts) {
            part_walk<R, ORDER2, PHI, CNT, SORTED_OUT, MAC, OCT>(
                nodes, m, bodies, anchors, perm, nbodies, t0 + 64 * g, kPartLanes * code, t1,
                theta2, eps2, acc, phi_out, npp_out, npc_out, gm);
            continue;
        }
        const bool fell = group_walk<R, ORDER2, PHI, CNT, SORTED_OUT, MAC, OCT>(
            nodes, m, bodies, anchors, kids, perm, nbodies, t0 + 64 * g, t1, theta2, eps2, acc,
            phi_out, npp_out, npc_out, gm, stk, stage, delta, level);
        if (gm.gfb && lane_id() == 0) {
            uint8_t *last = gm.gfb + ng;  // length of the group's last prediction
            if (fell) {
                const int len =
                    last[g] ? min(2 * (int)last[g], kPredictWalks) : gm.predict_first;
                last[g] = (uint8_t)len;
                gm.gfb[g] = (uint8_t)len;
            } else if (last[g]) {
                last[g] = 0;
            }
        }
    }
}

// Longest first.  A group of 64 consecutive bodies that straddles a jump of
// the space-filling curve has a box spanning the cells on both sides and
// costs many times an ordinary group; such groups are recognised by the
// smallest cell holding the group's first and last keys: the more bodies
// that cell holds, the more the group is spread out.  The cell is found
// from the tree, climbing from the first body's leaf to the first ancestor
// at or above the keys' common level (a cell holding more than a leaf's
// bodies is a node).  Within each XCD's chunk, groups predicted to exceed
// the work cap come first (kParts items each), then groups whose common
// cell holds more than 256 x 64 bodies, then those above 16 x 64, then the
// rest (order inside a class is immaterial: groups are independent).  Two
// launches over all groups: classify and count, then place.
//
// Queue memory per XCD chunk x (uint32 words at 64 x): [0] hand-out
// counter, [16] item count, [20 + c] items of class c, [24 + c] placed.
// hand-out position of a class: 3 first, then 0, 1, 2
__device__ __forceinline__ int class_pos(int c) { return c == 3 ? 0 : c + 1; }

template <typename R>
__device__ __forceinline__ int group_class(const uint64_t *__restrict__ keys, int t0, int t1,
                                           int g, const uint8_t *__restrict__ gfb,
                                           const Anchor<R> *__restrict__ anchors,
                                           const int32_t *__restrict__ level,
                                           const int32_t *__restrict__ parent,
                                           const int32_t *__restrict__ count) {
    if (gfb && gfb[g] > 0) return 3;
    const int r0 = t0 + 64 * g, r1 = min(r0 + 63, t1 - 1);
    const uint64_t x = keys[r0] ^ keys[r1];
    const int lcp = x == 0 ? 21 : (__builtin_clzll(x) - 1) / 3;  // shared octal digits
    int node = anchors[r0].leaf;
    for (int p; level[node] > lcp && (p = parent[node]) >= 0;) node = p;
    const int c = count[node];
    return c > 256 * 64 ? 0 : (c > 16 * 64 ? 1 : 2);
}

template <typename R>
__global__ __launch_bounds__(256) void k_group_class(const uint64_t *__restrict__ keys, int t0,
                                                     int t1, int ng,
                                                     const uint8_t *__restrict__ gfb,
                                                     const Anchor<R> *__restrict__ anchors,
                                                     const int32_t *__restrict__ level,
                                                     const int32_t *__restrict__ parent,
                                                     const int32_t *__restrict__ count,
                                                     uint8_t *__restrict__ cls,
                                                     uint32_t *__restrict__ queue) {
    __shared__ uint32_t cnt[8][4];  // per XCD chunk and class, this block's share
    if (threadIdx.x < 32) (&cnt[0][0])[threadIdx.x] = 0;
    __syncthreads();
    const int chunk = (ng + 7) / 8;
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g < ng) {
        const int c = group_class<R>(keys, t0, t1, g, gfb, anchors, level, parent, count);
        cls[g] = (uint8_t)c;
        atomicAdd(&cnt[g / chunk][c], c == 3 ? (uint32_t)kParts : 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const uint32_t v = (&cnt[0][0])[threadIdx.x];
        if (v) atomicAdd(&queue[64 * (threadIdx.x >> 2) + 20 + (threadIdx.x & 3)], v);
    }
}

__global__ __launch_bounds__(256) void k_group_place(int ng, const uint8_t *__restrict__ cls,
                                                     uint8_t *__restrict__ gfb,
                                                     uint32_t *__restrict__ items,
                                                     uint32_t *__restrict__ queue) {
    __shared__ uint32_t cnt[8][4], base[8][4];
    if (threadIdx.x < 32) (&cnt[0][0])[threadIdx.x] = 0;
    __syncthreads();
    const int chunk = (ng + 7) / 8;
    const int g = blockIdx.x * 256 + threadIdx.x;
    int c = 0, x = 0;
    uint32_t rank = 0;
    if (g < ng) {
        c = cls[g];
        x = g / chunk;
        rank = atomicAdd(&cnt[x][c], c == 3 ? (uint32_t)kParts : 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32) {  // reserve this block's range of every (chunk, class)
        const int xx = threadIdx.x >> 2, cc = threadIdx.x & 3;
        const uint32_t v = cnt[xx][cc];
        uint32_t b = 0;
        for (int k = 0; k < 4; ++k)
            if (class_pos(k) < class_pos(cc)) b += queue[64 * xx + 20 + k];
        base[xx][cc] = b + (v ? atomicAdd(&queue[64 * xx + 24 + cc], v) : 0u);
        if (blockIdx.x == 0 && cc == 0)
            queue[64 * xx + 16] = queue[64 * xx + 20] + queue[64 * xx + 21] +
                                  queue[64 * xx + 22] + queue[64 * xx + 23];
    }
    __syncthreads();
    if (g >= ng) return;
    uint32_t *out = items + kParts * (size_t)x * chunk;  // at most kParts items per group
    const uint32_t p = base[x][c] + rank;
    if (c == 3) {
        for (int q = 0; q < kParts; ++q) out[p + q] = (uint32_t)g * 16u + (uint32_t)q;
        gfb[g] = (uint8_t)(gfb[g] - 1);  // one prediction used up
    } else {
        out[p] = (uint32_t)g * 16u + kWholeGroup;
    }
}

__global__ void k_zero_bytes(uint8_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero_queue(uint32_t *q) { q[threadIdx.x] = 0u; }  // 512 threads

template <typename R, bool ORDER2, bool PHI, bool CNT, bool SORTED, int MAC, bool OCT>
void glaunch(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
             uint32_t *npp, uint32_t *npc, const GroupMac &gm, uint64_t sig) {
    // enough workgroups to fill every CU (8 per CU at this kernel's
    // register and LDS use), or fewer for small target ranges
    const int ng = div_up(t1 - t0, 64);
    const int per_xcd = std::min(div_up(div_up(ng, 8), 4), 256);
    uint32_t *queue = (uint32_t *)t->wq.p;
    k_zero_queue<<<1, 512, 0, t->ctx->stream>>>(queue);
    GroupMac g2 = gm;
    const int64_t waves = 8ll * per_xcd * 4;
    g2.predict_first = ng <= kLongPredictGroupsPerWave * waves ? kPredictWalks : 1;
    // fallback predictions hold for walks of this tree object with the same
    // parameters and targets (two bytes per group)
    uint8_t *gfb = nullptr;
    if (grow(t->gfb, 2ull * ng) == BH_OK) {
        gfb = (uint8_t *)t->gfb.p;
        if (t->gfb_sig != sig || t->gfb_ng != ng) {
            k_zero_bytes<<<std::min(div_up(2 * ng, 256), 1024), 256, 0, t->ctx->stream>>>(
                gfb, 2 * (int64_t)ng);
            t->gfb_sig = sig;
            t->gfb_ng = ng;
        }
    }
    // items (kParts slots per group), then one class byte per group
    if (grow(t->gorder, 4ull * kParts * ng + ng) == BH_OK) {
        uint32_t *items = (uint32_t *)t->gorder.p;
        uint8_t *cls = (uint8_t *)(items + (size_t)kParts * ng);
        k_group_class<R><<<div_up(ng, 256), 256, 0, t->ctx->stream>>>(
            t->sorted_keys, t0, t1, ng, gfb, (const Anchor<R> *)t->anchors.p,
            (const int32_t *)t->level.p, (const int32_t *)t->parent.p,
            (const int32_t *)t->count.p, cls, queue);
        k_group_place<<<div_up(ng, 256), 256, 0, t->ctx->stream>>>(ng, cls, gfb, items, queue);
        g2.items = items;
        g2.gfb = gfb;
    }
    if (t->ctx->walk_ev) hipEventRecord(t->ctx->walk_ev[0], t->ctx->stream);
    k_gwalk<R, ORDER2, PHI, CNT, SORTED, MAC, OCT><<<8 * per_xcd, 256, 0, t->ctx->stream>>>(
        (const typename NodeRecT<R>::type *)t->recs.p, (int)t->m,
        (const BodyRec<R> *)t->bodies.p, (const Anchor<R> *)t->anchors.p,
        (const int4 *)t->kids.p, t->perm, (int)t->n, t0, t1, queue, (R)(theta * theta),
        (R)(eps * eps), (R *)acc, (R *)phi, npp, npc, g2, (const int8_t *)t->delta.p,
        (const int32_t *)t->level.p);
    if (t->ctx->walk_ev) hipEventRecord(t->ctx->walk_ev[1], t->ctx->stream);
}

template <typename R, bool ORDER2, int MAC, bool OCT = false>
void gdispatch(bh_tree *t, int t0, int t1, double theta, double eps, void *acc, void *phi,
               uint32_t *npp, uint32_t *npc, bool sorted, const GroupMac &gm, uint64_t sig) {
    const bool P = phi != nullptr, C = npp != nullptr;
#define BH_G(p, c, s) glaunch<R, ORDER2, p, c, s, MAC, OCT>(t, t0, t1, theta, eps, acc, phi, npp, npc, gm, sig)
    if (sorted) {  // simulation walks: phi for the energy, counts when recorded
        if (P) BH_G(true, false, true);
        else if (C) BH_G(false, true, true);
        else BH_G(false, false, true);
    } else if (P && C) BH_G(true, true, false);
    else if (P) BH_G(true, false, false);
    else if (C) BH_G(false, true, false);
    else BH_G(false, false, false);
#undef BH_G
}

// group-walk state of the tree (the child table comes with every build)
int ensure_kids(bh_tree *t) {
    int rc = grow(t->wq, 8 * 256);  // group queue counters
    if (rc) return rc;
    if (t->kids_tree_id != t->build_id) return set_error(BH_E_STATE, "tree has no child table");
    return BH_OK;
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
    t->last_mac = o.mac;
    if (o.n_pq && !npp && !npc) {  // the quadrupole terms are counted with the others
        int rc = grow(t->cnt_scratch, 8ull * t->n);
        if (rc) return rc;
        npp = (uint32_t *)t->cnt_scratch.p;
        npc = npp + t->n;
    } else if ((npp != nullptr) != (npc != nullptr)) {  // the kernel writes both or neither
        int rc = grow(t->cnt_scratch, 4ull * t->n);
        if (rc) return rc;
        if (!npp) npp = (uint32_t *)t->cnt_scratch.p;
        else npc = (uint32_t *)t->cnt_scratch.p;
    }
    MlpMac mac{nullptr, nullptr, nullptr, 0.f, 0.f};
    mac.npq = o.n_pq;
    const bool group = o.walk == BH_WALK_GROUP;
    if (group) {
        int rc = ensure_kids(t);
        if (rc) return rc;
    }
    GroupMac gm{nullptr, nullptr, nullptr, 0.f, o.walk_stack > 0 ? o.walk_stack : kGroupStack,
                o.walk_cap > 0                 ? o.walk_cap
                : o.mac == BH_MAC_BUDGET       ? kGroupWorkCapBudget
                                               : kGroupWorkCap,
                nullptr, nullptr, kPredictWalks};
    gm.npq = o.n_pq;
    // the parameters that decide which groups exceed the work cap (FNV-1a)
    uint64_t sig = 1469598103934665603ull;
    auto mixin = [&](const void *p, size_t len) {
        for (size_t k = 0; k < len; ++k) {
            sig ^= ((const unsigned char *)p)[k];
            sig *= 1099511628211ull;
        }
    };
    {
        const double dv[6] = {theta, eps, o.mlp_theta_max, o.mlp_log10_tau, o.mlp_acc_floor,
                              (double)o.walk_cap};
        const int64_t iv[7] = {o.mac, o.order, t0, t1, t->dtype,
                               o.mac == BH_MAC_MLP ? t->ctx->mlp_version : 0,
                               o.mac == BH_MAC_MLP ? o.mlp_precision : 0};
        mixin(dv, sizeof dv);
        mixin(iv, sizeof iv);
        sig |= 1ull << 63;  // never the unset value 0
    }
    if (o.mac == BH_MAC_MLP || o.mac == BH_MAC_BUDGET) {
        const bool learned = o.mac == BH_MAC_MLP;
        if (t->dtype != BH_F32 || (o.order != 2 && (learned || o.order > 2)))
            return set_error(BH_E_INVALID, learned
                                               ? "the learned criterion runs in the FP32 quadrupole walk"
                                               : "the error budget runs in the FP32 walk of order 0, 1 (mixed) or 2");
        const bool mono = o.order == 0, mixed = o.order == BH_ORDER_MIXED;
        int rc = learned ? BH_OK : mlp_cells(t);
        if (rc) return rc;
        if (o.mlp_acc_norm) {
            rc = mlp_anorm(t, nullptr, o.mlp_acc_norm, true, o.mlp_acc_floor);
        } else if (prev_acc) {
            rc = mlp_anorm(t, prev_acc, nullptr, true, o.mlp_acc_floor);
        } else {
            // estimate |a_i| of the targets with a monopole walk at theta_est
            if ((rc = grow(t->est_acc, 12ull * t->n))) return rc;
            bh_force_opts eo;
            bh_force_opts_default(&eo);
            eo.order = 0;
            eo.walk = o.walk;
            eo.walk_stack = o.walk_stack;
            eo.walk_cap = o.walk_cap;
            eo.target_begin = t0;
            eo.target_end = t1;
            if ((rc = run_walk(t, o.mlp_theta_est, eps, t->est_acc.p, nullptr, nullptr, nullptr, eo,
                               true)))
                return rc;
            rc = mlp_anorm(t, t->est_acc.p, nullptr, false, o.mlp_acc_floor);
        }
        if (rc) return rc;
        mac.kc = learned ? nullptr : (const float *)t->kc.p;
        mac.anorm = (const float *)t->anorm.p;
        mac.afloor = mlp_anorm_floor(t);
        mac.tmax2 = (float)(o.mlp_theta_max * o.mlp_theta_max);
        mac.tau = (float)pow(10.0, o.mlp_log10_tau);
        mac.net = learned ? (const MlpPacked *)t->ctx->mlp_w.p + o.mlp_precision : nullptr;
        mac.eps = (float)eps;
        const bool f16 = o.mlp_precision == BH_MLP_FP16;
        if (group) {
            gm.kc = mac.kc;
            gm.anorm = mac.anorm;
            gm.afloor = mac.afloor;
            gm.tau = mac.tau;
            gm.net = mac.net;
            gm.eps = mac.eps;
#define BH_GM(k) gdispatch<float, true, k>(t, t0, t1, o.mlp_theta_max, eps, acc, phi, npp, npc, sorted_out, gm, sig)
            if (!learned && mono) gdispatch<float, false, 1>(t, t0, t1, o.mlp_theta_max, eps, acc, phi, npp, npc, sorted_out, gm, sig);
            else if (!learned && mixed) BH_GM(4);
            else if (!learned) BH_GM(1);
            else if (f16) BH_GM(3);
            else BH_GM(2);
#undef BH_GM
        } else {
#define BH_BM(k) dispatch2<float, true, k>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac)
            if (!learned && mono) dispatch2<float, false, 1>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
            else if (!learned && mixed) BH_BM(4);
            else if (!learned) BH_BM(1);
            else if (f16) BH_BM(3);
            else BH_BM(2);
#undef BH_BM
        }
    } else if (o.order == 3) {  // the opening angle with the octopole term
        int rc = ensure_octopole(t);
        if (rc) return rc;
        gm.oct = mac.oct = t->oct.p;
        if (group) {
            if (t->dtype == BH_F32) gdispatch<float, true, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
            else gdispatch<double, true, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
        } else {
            if (t->dtype == BH_F32) dispatch2<float, true, 0, false, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
            else dispatch2<double, true, 0, false, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        }
    } else if (group) {
        if (t->dtype == BH_F32) {
            if (o.order == 0) gdispatch<float, false, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
            else gdispatch<float, true, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
        } else {
            if (o.order == 0) gdispatch<double, false, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
            else gdispatch<double, true, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, gm, sig);
        }
    } else if (o.mac == BH_MAC_THETA_GUARD) {  // per-body walk only (checked by the caller)
        if (t->dtype == BH_F32) {
            if (o.order == 0) dispatch2<float, false, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
            else dispatch2<float, true, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        } else {
            if (o.order == 0) dispatch2<double, false, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
            else dispatch2<double, true, 0, true>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        }
    } else if (t->dtype == BH_F32) {
        if (o.order == 0) dispatch2<float, false, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        else dispatch2<float, true, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
    } else {
        if (o.order == 0) dispatch2<double, false, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
        else dispatch2<double, true, 0>(t, t0, t1, theta, eps, acc, phi, npp, npc, sorted_out, mac);
    }
    return check_launch("walk");
}

}  // namespace bh
