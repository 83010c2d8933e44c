// The interleaved FK + collision walk and the persistent edge launch, as device code that both
// the library's kernels (vk_kernels.hip, one kernel for every robot) and the per-robot kernels
// compiled at run time (vk_robot_specialize) include.  It uses no host headers, so the runtime
// compiler can take it as it is.
#pragma once
#include <stdint.h>

#include <type_traits>

#include "vk_device.hpp"

namespace vk {

// The robot program and the batch descriptors are never written while a kernel runs.  Reading
// them through the constant address space lets every wave-uniform access compile to a scalar
// load; through a generic pointer the stores elsewhere in a kernel (flags, queue) can force
// vector loads of uniform data.  A record is copied word by word and unused words fold away.
template <class T>
__device__ __forceinline__ T ld(const T *p, int64_t i) {
    static_assert(sizeof(T) % 4 == 0, "records are whole words");
    T out;
    const __attribute__((address_space(4))) uint32_t *src =
        (const __attribute__((address_space(4))) uint32_t *)(p + i);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(T) / 4); ++w) dst[w] = src[w];
    return out;
}

// Value of the first active lane, as a wave-uniform 64-bit integer.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)v);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Robot program sources.  DynProg reads the records the host built for a robot with
// wave-uniform scalar loads: one compiled kernel serves every robot.  SpecProg<R> reads them
// from the constant arrays of a struct R generated for one robot and compiled at run time
// (vk_robot_specialize): with every field known at compile time, the per-step code (posing,
// placement, the self-pair blocks and their entries) unrolls with its constants folded into
// the instructions and its loads gone, the GPU form of the straight-line code that the paper's
// tracing compiler generates per robot (Sec. III-B).
struct DynProg {
    const RobotDev &rb;
    static constexpr bool kSpec = false;
    __device__ __forceinline__ int n_steps() const { return rb.n_steps; }
    __device__ __forceinline__ int dof() const { return rb.dof; }
    __device__ __forceinline__ StepRec step(int i) const { return ld(rb.steps, i); }
    __device__ __forceinline__ BlockRec block(int i) const { return ld(rb.blocks, i); }
    __device__ __forceinline__ EntryRec entry(int i) const { return ld(rb.entries, i); }
    __device__ __forceinline__ JointRec path_rec(int i) const { return ld(rb.path_recs, i); }
    __device__ __forceinline__ float4 sphere(int i) const { return ld(rb.spheres, i); }
    // run f for step st (a value known at run time)
    template <class F>
    __device__ __forceinline__ int at_step(int st, F &&f) const { return f(st); }
};

// R provides dof, n_steps, and constant arrays steps[], blocks[], entries[], path_recs[] and
// spheres[] (the records DynProg would load).
template <class R>
struct SpecProg {
    const RobotDev &rb;
    static constexpr bool kSpec = true;
    __device__ __forceinline__ int n_steps() const { return R::n_steps; }
    __device__ __forceinline__ int dof() const { return R::dof; }
    // A record's integer fields (counts, indices, codes, masks) come from the constant array, so
    // with a compile-time index they fold into the control flow; its float fields are loaded
    // where they are used, through a pointer the compiler cannot see through.  gfx950's
    // three-operand vector instructions take no literal operands, so folded float constants
    // would each need a register, and the compiler hoists them out of the walk's loops: loading
    // them keeps their live ranges as short as the interpreted walk's.
    template <class T>
    __device__ __forceinline__ static const T *opaque(const T *p) {
        asm volatile("" : "+s"(p));
        return p;
    }
    __device__ __forceinline__ static JointRec joint_mix(JointRec c, const JointRec &v) {
        c.a = v.a;
        c.d = v.d;
        c.ca = v.ca;
        c.sa = v.sa;
        c.theta_off = v.theta_off;
        c.s_off = v.s_off;
        c.c_off = v.c_off;
#pragma unroll
        for (int k = 0; k < 12; ++k) c.m[k] = v.m[k];
        return c;
    }
    __device__ __forceinline__ StepRec step(int i) const {
        StepRec c = R::steps[i];
        const StepRec v = ld(opaque(R::steps), i);
#pragma unroll
        for (int k = 0; k < 4; ++k) c.coarse[k] = v.coarse[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) c.cap_h[k] = v.cap_h[k];
        c.cap_r = v.cap_r;
        c.cap_rq = v.cap_rq;
        c.cap_uu = v.cap_uu;
        c.cap_inv = v.cap_inv;
        c.jr = joint_mix(c.jr, v.jr);
        return c;
    }
    __device__ __forceinline__ BlockRec block(int i) const {
        BlockRec c = R::blocks[i];
        const BlockRec v = ld(opaque(R::blocks), i);
        c.ra = v.ra;
        c.rqa = v.rqa;
        return c;
    }
    __device__ __forceinline__ EntryRec entry(int i) const {
        EntryRec c = R::entries[i];
        const EntryRec v = ld(opaque(R::entries), i);
        c.x = v.x;
        c.y = v.y;
        c.z = v.z;
        c.r = v.r;
        c.gate2 = v.gate2;
        c.nhr2 = v.nhr2;
#pragma unroll
        for (int k = 0; k < kSpl; ++k) c.rr[k] = v.rr[k];
        return c;
    }
    __device__ __forceinline__ JointRec path_rec(int i) const {
        return joint_mix(R::path_recs[i], ld(opaque(R::path_recs), i));
    }
    __device__ __forceinline__ float4 sphere(int i) const { return ld(opaque(R::spheres), i); }
    // run f with step st as a compile-time constant (a chain of uniform compares)
    template <int I, class F>
    __device__ __forceinline__ int dispatch(int st, F &f) const {
        if constexpr (I + 1 >= R::n_steps) {
            return f(std::integral_constant<int, I>());
        } else {
            if (st == I) return f(std::integral_constant<int, I>());
            return dispatch<I + 1>(st, f);
        }
    }
    // Each call site hides st from the optimizer: otherwise it threads the successive
    // dispatches of one step through the code between them, copying the whole environment part
    // once per step.
    template <class F>
    __device__ __forceinline__ int at_step(int st, F &&f) const {
        asm volatile("" : "+s"(st));
        return dispatch<0>(st, f);
    }
};

// for (i = 0; i < n; ++i) if (f(i)) break; -- fully unrolled for a specialised program (n is
// then a constant), a plain loop otherwise.
template <class P, class F>
__device__ __forceinline__ void for_n(int n, F &&f) {
    if constexpr (P::kSpec) {
#pragma unroll
        for (int i = 0; i < n; ++i)
            if (f(i)) break;
    } else {
        for (int i = 0; i < n; ++i)
            if (f(i)) break;
    }
}

// Joint value sources ------------------------------------------------------------------------
struct QEdge {                 // state on a straight edge: qa + t (qb - qa), qa/qb uniform
    const float *a;            // (t = 1 gives qb exactly, so both endpoints are the inputs)
    const float *b;
    float t;
    __device__ __forceinline__ float operator()(int j) const {
        const float x = ld(a, j), y = ld(b, j);
        return t == 1.0f ? y : fmaf(t, y - x, x);
    }
};

struct QState {                // SoA state batch: q[j * ldq + i]
    const float *q;
    int64_t ldq;
    int64_t i;
    __device__ __forceinline__ float operator()(int j) const { return q[j * ldq + i]; }
};

// Environment view (records in LDS or global memory) -----------------------------------------
struct EnvView {
    const float4 *rec;             // primitive records
    const float *cell;             // point-grid cell index (int bits)
    int off_sph, off_cap, off_cyl, off_box;
    int n_sph, n_cap, n_cyl, n_box;
};

// Staging modes of the record buffer: 0 nothing in LDS, 1 the primitives, 2 the primitives and
// the point-grid cell index.  `lds` holds the staged prefix.  The mode is a template constant so
// that every record access compiles to an LDS or a global load, never a generic one.
template <int STAGE>
__device__ __forceinline__ EnvView make_view(const EnvDev &e, const float4 *lds) {
    EnvView v;
    v.rec = STAGE ? lds : e.rec;
    v.cell = reinterpret_cast<const float *>((STAGE == 2 ? lds : e.rec) + e.off_cell);
    v.off_sph = e.off_sph;
    v.off_cap = e.off_cap;
    v.off_cyl = e.off_cyl;
    v.off_box = e.off_box;
    v.n_sph = e.n_sph;
    v.n_cap = e.n_cap;
    v.n_cyl = e.n_cyl;
    v.n_box = e.n_box;
    return v;
}

// Overlap of sphere (x, y, z, r) with primitive `i` of type `t` (0 sphere, 1 capsule,
// 2 cylinder, 3 box), records read from the view.
__device__ __forceinline__ bool hit_any(const EnvView &ev, int t, int i, float x, float y,
                                        float z, float r) {
    if (t == 3) {
        const float4 *b = ev.rec + ev.off_box + 4 * i;
        return hit_box(x, y, z, r, b[0], b[1], b[2], b[3]);
    }
    if (t == 1) {
        const float4 *c = ev.rec + ev.off_cap + 2 * i;
        return hit_capsule(x, y, z, r, c[0], c[1]);
    }
    if (t == 0) return hit_sphere(x, y, z, r, ev.rec[ev.off_sph + i]);
    const float4 *c = ev.rec + ev.off_cyl + 2 * i;
    return hit_cylinder(x, y, z, r, c[0], c[1]);
}

// Signed distance and gradient to primitive `i` of type `t`.
__device__ __forceinline__ float sd_any(const EnvView &ev, int t, int i, float x, float y, float z,
                                        float &gx, float &gy, float &gz) {
    if (t == 3) {
        const float4 *b = ev.rec + ev.off_box + 4 * i;
        return sd_box(x, y, z, b[0], b[1], b[2], b[3], gx, gy, gz);
    }
    if (t == 1) {
        const float4 *c = ev.rec + ev.off_cap + 2 * i;
        return sd_capsule(x, y, z, c[0], c[1], gx, gy, gz);
    }
    if (t == 0) return sd_sphere(x, y, z, ev.rec[ev.off_sph + i], gx, gy, gz);
    const float4 *c = ev.rec + ev.off_cyl + 2 * i;
    return sd_cylinder(x, y, z, c[0], c[1], gx, gy, gz);
}

// Voxel broadphase lookup for a link bounding sphere (C, CR <= vcap): the candidate range
// [b, e) of the cell holding C, empty when the cell's smallest lower bound is >= CR or C lies
// outside the grid (then nothing is within vcap of C).
__device__ __forceinline__ void voxel_range(const EnvView &ev, const EnvDev &ed, float Cx,
                                            float Cy, float Cz, float CR, int &b, int &e) {
    b = e = 0;
    const float fx = floorf((Cx - ed.vorg[0]) * ed.vinv);
    const float fy = floorf((Cy - ed.vorg[1]) * ed.vinv);
    const float fz = floorf((Cz - ed.vorg[2]) * ed.vinv);
    if (!(fx >= 0.0f && fy >= 0.0f && fz >= 0.0f && fx < (float)ed.vdim[0] &&
          fy < (float)ed.vdim[1] && fz < (float)ed.vdim[2]))
        return;
    const int cell = ((int)fz * ed.vdim[1] + (int)fy) * ed.vdim[0] + (int)fx;
    const unsigned char *dist = reinterpret_cast<const unsigned char *>(ed.rec + ed.off_vdist);
    if ((float)dist[cell] * ed.vq >= CR) return;
    b = ed.vstart[cell];
    e = ed.vstart[cell + 1];
}

// Copy the environment records into LDS once per workgroup.
__device__ __forceinline__ void stage_env(float4 *lds, const float4 *__restrict__ g, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
    __syncthreads();
}

// Executed-work accounting (FLOP model, FMA = 2): every wave-uniform operation below adds its
// per-lane FLOP count; the instrumented kernel multiplies by the 64 lanes that issue it.
// NoWork compiles to nothing, so the timed kernels carry no accounting.
// The method's own work is split in four categories: FK and sphere placement, culling (voxel
// lookups and per-link bounding-sphere tests), fine environment tests, self pairs (their gates
// and tests).  Two more categories hold work this implementation adds to the method: re-posing
// (posing an earlier link again for a self block, rebuilding a tree branch, placing the earlier
// link's spheres again), and surplus rake lanes (the lanes an edge of fewer than 64 * steps
// states leaves over repeat its last state; everything they execute goes here).  Every lane
// counts the operations it executes (lanes masked off by divergent control flow add nothing);
// the instrumented kernel sums the lanes.  `visits` counts the rake slots of real states that a
// lane walks (whatever the walk's length): the rake schedule and its early exit alone decide it.
namespace flop {
constexpr uint32_t kJoint = 30, kMount = 63, kPlace = 18, kSphere = 11, kCapsule = 25,
                   kCylinder = 35, kBox = 34, kPair = 11;
// capsule bound against capsule bound (unpacking the earlier one and the segment distance),
// sphere bound against capsule bound, and rotating a step's capsule half-vector to the world frame
constexpr uint32_t kCapsuleCapsule = 67, kSphereCapsule = 28, kPlaceHalf = 15;
// looking up a location in the point-cloud clearance field (cell index, the distance to the
// cell's centre, the bound)
constexpr uint32_t kClearance = 23;
enum Cat { kFk = 0, kCull = 1, kFine = 2, kSelf = 3, kRepose = 4, kSurplus = 5, kCats = 6 };
}
struct NoWork {
    __device__ __forceinline__ void add(int, uint32_t) {}
    __device__ __forceinline__ void rake_slot(bool) {}
};
struct Work {
    uint64_t f[flop::kCats] = {0, 0, 0, 0, 0, 0};
    uint64_t visits = 0;
    bool surplus = false;
    __device__ __forceinline__ void add(int c, uint32_t x) { f[surplus ? flop::kSurplus : c] += x; }
    // a rake slot begins: a real state of the edge, or a surplus lane repeating the last one
    __device__ __forceinline__ void rake_slot(bool real) {
        surplus = !real;
        visits += real ? 1 : 0;
    }
};

// Per-wave LDS cache, per lane, with a slot for each step whose bounds a later self block
// reads: the world centre of the step's link bounding sphere ([slot][axis][lane]), optionally
// the world half-vector of its bounding capsule as three halves ([slot][2][lane], after the
// centres), and optionally the sine and cosine of every joint angle ([joint][2][lane], after
// those), all written by the walk as it poses each link.  The centres
// and capsules gate self blocks without posing the earlier link; the joint sines and cosines
// make re-posing an earlier link (and rebuilding a tree branch) cost the DH products only.
typedef __fp16 half2_t __attribute__((ext_vector_type(2)));

struct StepCache {
    float *base;
    int lane;
    int half_off;                  // n_slots * 3 * kWave, or -1 without the capsule halves
    int joint_off;                 // after the centres and halves, or -1 without the joint slots
    __device__ __forceinline__ void put(int st, float x, float y, float z) const {
        base[(st * 3 + 0) * kWave + lane] = x;
        base[(st * 3 + 1) * kWave + lane] = y;
        base[(st * 3 + 2) * kWave + lane] = z;
    }
    __device__ __forceinline__ void get(int st, float &x, float &y, float &z) const {
        x = base[(st * 3 + 0) * kWave + lane];
        y = base[(st * 3 + 1) * kWave + lane];
        z = base[(st * 3 + 2) * kWave + lane];
    }
    // capsule half-vector, each component rounded toward zero to half precision
    __device__ __forceinline__ void put_h(int st, float x, float y, float z) const {
        base[half_off + (st * 2 + 0) * kWave + lane] =
            __builtin_bit_cast(float, __builtin_amdgcn_cvt_pkrtz(x, y));
        base[half_off + (st * 2 + 1) * kWave + lane] =
            __builtin_bit_cast(float, __builtin_amdgcn_cvt_pkrtz(z, 0.0f));
    }
    __device__ __forceinline__ void get_h(int st, float &x, float &y, float &z) const {
        const half2_t u = __builtin_bit_cast(half2_t, base[half_off + (st * 2 + 0) * kWave + lane]);
        const half2_t w = __builtin_bit_cast(half2_t, base[half_off + (st * 2 + 1) * kWave + lane]);
        x = (float)u.x;
        y = (float)u.y;
        z = (float)w.x;
    }
    // joint values: (sin, cos) of a revolute joint's angle, (offset, unused) of a prismatic one
    __device__ __forceinline__ void put_val(int j, const JointRec &J, const JointVal &v) const {
        base[joint_off + (j * 2 + 0) * kWave + lane] = J.prismatic ? v.d : v.s;
        base[joint_off + (j * 2 + 1) * kWave + lane] = v.c;
    }
    __device__ __forceinline__ JointVal get_val(int j, const JointRec &J) const {
        const float u = base[joint_off + (j * 2 + 0) * kWave + lane];
        const float w = base[joint_off + (j * 2 + 1) * kWave + lane];
        JointVal v;
        if (J.prismatic) {
            v.s = J.s_off;
            v.c = J.c_off;
            v.d = u;
        } else {
            v.s = u;
            v.c = w;
            v.d = J.d;
        }
        return v;
    }
};

__device__ __forceinline__ StepCache make_step_cache(float *base, int n_slots, int cf) {
    const int words = (cf & kCacheCaps) ? 5 : 3;
    return StepCache{base, (int)(threadIdx.x & (kWave - 1)),
                     (cf & kCacheCaps) ? n_slots * 3 * kWave : -1,
                     (cf & kCacheJoints) ? n_slots * words * kWave : -1};
}

// Dynamic LDS of the walks: [cache of every wave of the block][environment records].
__device__ __forceinline__ StepCache step_cache(float *lds, int n_slots, int dof, int cf) {
    return make_step_cache(lds + (threadIdx.x / kWave) * step_cache_floats(n_slots, dof, cf),
                           n_slots, cf);
}
__device__ __forceinline__ float4 *after_caches(float *lds, int n_slots, int dof, int cf) {
    return reinterpret_cast<float4 *>(lds + (blockDim.x / kWave) * step_cache_floats(n_slots, dof, cf));
}

// Pose the link of step S into T (rebuilding a tree branch from the base when needed).  With a
// cache, the step's joint keeps its sine and cosine there and a rebuilt branch reads the
// earlier joints' values back instead of evaluating them again.
template <class P, class Q, class W = NoWork>
__device__ __forceinline__ void pose_step(const P &pg, const StepRec &S, Frame &T,
                                          const Q &q, W &&w = W(),
                                          const StepCache *sc = nullptr) {
    if (S.joint < 0) return;
    if (S.restart_len >= 0) {
        frame_identity(T);
        for_n<P>(S.restart_len, [&](int k) __attribute__((always_inline)) {
            const JointRec J = pg.path_rec(S.restart_off + k);
            const int j = J.index;
            if (sc && sc->joint_off >= 0)
                frame_joint_val(T, J, sc->get_val(j, J));
            else
                frame_joint(T, J, q(j));
            w.add(flop::kRepose, flop::kJoint + (J.has_mount ? flop::kMount : 0));
            return false;
        });
    }
    const JointRec &J = S.jr;
    const JointVal v = joint_val(J, q(S.joint));
    if (sc && sc->joint_off >= 0) sc->put_val(S.joint, J, v);
    frame_joint_val(T, J, v);
    w.add(flop::kFk, flop::kJoint + (J.has_mount ? flop::kMount : 0));
}

// Pose the earlier link A of self block B into Ta, from the cached joint sines and cosines when
// the cache has them (every joint on A's path was evaluated by the walk before).  Ta holds link
// `ta_link` (depth `ta_depth` joints from the base): when that link is A nothing is done; when
// it is the base or a proper ancestor of A the remaining joints of A's path are applied;
// otherwise Ta restarts from the base.
template <class P, class Q, class W = NoWork>
__device__ __forceinline__ void pose_block(const P &pg, const BlockRec &B, Frame &Ta,
                                           int &ta_link, int &ta_depth, const StepCache &sc,
                                           const Q &q, W &&w = W()) {
    if (ta_link == B.link) return;
    const unsigned long long anc = ((unsigned long long)B.anc_hi << 32) | B.anc_lo;
    int k0 = ta_depth;
    if (!(ta_link == 0 || (ta_link > 0 && ((anc >> (ta_link - 1)) & 1ull)))) {
        frame_identity(Ta);
        k0 = 0;
    }
    const auto joint = [&](int k) __attribute__((always_inline)) {
        const JointRec J = pg.path_rec(B.path_off + k);
        const int j = J.index;
        if (sc.joint_off >= 0)
            frame_joint_val(Ta, J, sc.get_val(j, J));
        else
            frame_joint(Ta, J, q(j));
        w.add(flop::kRepose, flop::kJoint + (J.has_mount ? flop::kMount : 0));
    };
    for (int k = k0; k < B.path_len; ++k) joint(k);
    ta_link = B.link;
    ta_depth = B.path_len;
}

// Sphere centres of a step from its link frame (placed lazily, when a test needs them).  All
// kSpl slots are loaded and placed without branches (the sphere array carries kSpl records of
// padding): slots k >= sph_count hold finite values with radius 0 and every consumer either
// skips them or, in the self test, neutralises them with a -inf pair constant.
template <class P>
__device__ __forceinline__ void place_step(const P &pg, const StepRec &S, const Frame &T,
                                           float (&cx)[kSpl], float (&cy)[kSpl],
                                           float (&cz)[kSpl], float (&cr)[kSpl]) {
    float4 sv[kSpl];
#pragma unroll
    for (int k = 0; k < kSpl; ++k) sv[k] = pg.sphere(S.sph_first + k);
#pragma unroll
    for (int k = 0; k < kSpl; ++k) {
        if (P::kSpec && k >= S.sph_count) {   // a specialised program skips the padding slots
            cx[k] = cy[k] = cz[k] = cr[k] = 0.0f;
            continue;
        }
        frame_point(T, sv[k].x, sv[k].y, sv[k].z, cx[k], cy[k], cz[k]);
        cr[k] = k < S.sph_count ? sv[k].w : 0.0f;
    }
}


// Grid broadphase over a large set of small spheres.  A point of radius <= gmax_r can touch a
// robot sphere (c, r) only if its centre lies within r + gmax_r of c, i.e. in one of the cells
// that the box c -+ (r + gmax_r) touches; the cells of one row are contiguous in the sorted
// point array, so each (z, y) row of that box is one contiguous range [b, e) of it.
// `row(b, e)` returns true to stop.  With AHEAD the next row's bounds are loaded before the
// current row is visited (for the wave-wide scan, where they are scalar loads).
template <bool AHEAD = false, class F>
__device__ __forceinline__ void grid_rows(const EnvView &ev, const GridDev &g, float cx, float cy,
                                          float cz, float r, F &&row) {
    const float *cell = ev.cell;
    // the cells that the box c -+ (r + largest point radius) touches (widened a little for the
    // float rounding of the cell coordinates)
    const float reach = (r + g.gmax_r) * 1.00001f + 1e-5f, lim = 1.0e6f;
    const auto lo = [&](float c, float o) {
        return max((int)fminf(fmaxf(floorf((c - reach - o) * g.ginv), -lim), lim), 0);
    };
    const auto hi = [&](float c, float o, int n) {
        return min((int)fminf(fmaxf(floorf((c + reach - o) * g.ginv), -lim), lim), n - 1);
    };
    const int x0 = lo(cx, g.gorg[0]), x1 = hi(cx, g.gorg[0], g.gdim[0]);
    const int y0 = lo(cy, g.gorg[1]), y1 = hi(cy, g.gorg[1], g.gdim[1]);
    const int z0 = lo(cz, g.gorg[2]), z1 = hi(cz, g.gorg[2], g.gdim[2]);
    if (x0 > x1) return;
    if (!AHEAD) {
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) {
                const int rw = (z * g.gdim[1] + y) * g.gdim[0];
                if (row(__float_as_int(cell[rw + x0]), __float_as_int(cell[rw + x1 + 1]))) return;
            }
        return;
    }
    if (y0 > y1 || z0 > z1) return;
    int z = z0, y = y0, rw = (z0 * g.gdim[1] + y0) * g.gdim[0];
    int nb = __float_as_int(cell[rw + x0]), ne = __float_as_int(cell[rw + x1 + 1]);
    for (;;) {
        const int b = nb, e = ne;
        if (++y > y1) {
            y = y0;
            ++z;
        }
        const bool more = z <= z1;
        if (more) {
            rw = (z * g.gdim[1] + y) * g.gdim[0];
            nb = __float_as_int(cell[rw + x0]);
            ne = __float_as_int(cell[rw + x1 + 1]);
        }
        if (row(b, e) || !more) return;
    }
}

// Lower bound of the clearance of location (x, y, z) to every point of the grid: the field's
// value at the centre of the cell holding the location, less the distance to that centre
// (clearance changes by at most the distance moved, so the bound holds whichever cell FP32
// rounding picks); a location outside the field is at least 255 units away.
__device__ __forceinline__ float point_clearance(const GridDev &g, float x, float y, float z) {
    const float lim = 1.0e6f;
    const int ix = (int)fminf(fmaxf(floorf((x - g.porg[0]) * g.pinv), -lim), lim);
    const int iy = (int)fminf(fmaxf(floorf((y - g.porg[1]) * g.pinv), -lim), lim);
    const int iz = (int)fminf(fmaxf(floorf((z - g.porg[2]) * g.pinv), -lim), lim);
    const bool in = ix >= 0 && iy >= 0 && iz >= 0 && ix < g.pdim[0] && iy < g.pdim[1] &&
                    iz < g.pdim[2];
    if (!in) return 255.0f * g.pq;
    const float dx = x - fmaf((float)ix + 0.5f, g.pcell, g.porg[0]);
    const float dy = y - fmaf((float)iy + 0.5f, g.pcell, g.porg[1]);
    const float dz = z - fmaf((float)iz + 0.5f, g.pcell, g.porg[2]);
    const float v = (float)g.pfield[(iz * g.pdim[1] + iy) * g.pdim[0] + ix] * g.pq;
    return v - sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
}

// Does sphere (c, r) touch a point of the grid?  Per lane: a row's points are read kGridBatch
// at a time, so that a lane waits for one round of loads per batch rather than per point (the
// loads past the row's end repeat its last point; the answer is the same whichever order finds
// the hit).  Three: with four or more in flight the walk kernels spilled over a hundred
// registers.
constexpr int kGridBatch = 3;
__device__ __forceinline__ bool grid_hit(const EnvView &ev, const GridDev &g, float cx, float cy,
                                         float cz, float r) {
    bool hit = false;
    grid_rows(ev, g, cx, cy, cz, r, [&](int b, int e) {
        for (int p = b; p < e; p += kGridBatch) {
            float4 o[kGridBatch];
#pragma unroll
            for (int u = 0; u < kGridBatch; ++u) o[u] = g.pts[min(p + u, e - 1)];
#pragma unroll
            for (int u = 0; u < kGridBatch; ++u) hit |= hit_sphere(cx, cy, cz, r, o[u]);
            if (hit) return true;
        }
        return false;
    });
    return hit;
}

// The same test for a sphere that every lane holds (wave-uniform c, r): the lanes read 64
// consecutive points of a row at a time.  Called in wave-uniform control flow with every lane
// of the wave active; the answer is wave-uniform.
__device__ __forceinline__ bool grid_hit_wave(const EnvView &ev, const GridDev &g, float cx,
                                              float cy, float cz, float r) {
    const int lane = threadIdx.x & (kWave - 1);
    bool hit = false;
    grid_rows<true>(ev, g, cx, cy, cz, r, [&](int b, int e) {
        for (int p0 = b; p0 < e; p0 += kWave) {
            const int p = min(p0 + lane, e - 1);
            if (wave_ballot(hit_sphere(cx, cy, cz, r, g.pts[p]))) {
                hit = true;
                return true;
            }
        }
        return false;
    });
    return hit;
}

// Sum over the wave's 64 lanes, the same value (bit for bit) in every lane.
__device__ __forceinline__ float wave_sum(float v) {
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

// One lane's value, wave-uniform.
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Gated fine test: the step's bounding sphere (coarse) must touch the primitive in some live
// lane before the step's spheres are tested against it; then the exit test.
#define VK_GATE(KFLOP, COARSE, FINE)                                                \
    work.add(flop::kCull, KFLOP);                                                   \
    if (wave_ballot(live && (COARSE))) {                                            \
        work.add(flop::kFine, (KFLOP) * cnt);                                       \
        _Pragma("unroll") for (int k = 0; k < kSpl; ++k) if (k < cnt) col |= (FINE); \
        if (EDGE) {                                                                 \
            if (wave_ballot(col)) return true;                                      \
        } else {                                                                    \
            live = !col;                                                            \
            if (!wave_ballot(live)) return col;                                     \
        }                                                                           \
    }

// The interleaved FK + collision walk of one configuration per lane.
//   EDGE = true : returns as soon as any lane of the wave collides (the edge is invalid); the
//                 return value is then wave-uniform.
//   EDGE = false: per-lane result; lanes that collided stop contributing, and the walk ends
//                 when every lane has collided.  `col` on entry marks lanes already decided.
// With RANGED only the tests numbered [test_from, test_to) run, else all of them.  The tests
// are numbered in walk order: step s's environment part is number s + blk_first(s), its self
// blocks follow it (blocks are numbered across steps in step order).  Steps before the range
// are posed and cached only, and the walk stops before the first step past it.
// The step loop is a loop at run time.  The parts that depend on the step's records (posing and
// caching the link, placing its spheres, its self-pair blocks) go through pg.at_step, which for
// a robot-specialised program selects code compiled for that step with its records as
// constants; the environment part, which depends on the records only through a few values,
// exists once.
template <bool EDGE, bool RANGED = !EDGE, class P, class Q, class W = NoWork>
__device__ __forceinline__ bool walk_collide(const P &pg, const EnvView &ev, const EnvDev &ed, const Q &q,
                             const StepCache &sc, bool col, int test_from, int test_to,
                             W &&work = W()) {
    Frame Tm, Ta;
    frame_identity(Tm);
    frame_identity(Ta);
    int ta_link = 0, ta_depth = 0;
    bool live = !col;
    if (!EDGE && !wave_ballot(live)) return col;
    const int n_steps = pg.n_steps();
    for (int st = 0; st < n_steps; ++st) {
        // pose the step's link, cache its bounds; the values the environment part reads
        int cnt = 0, ibase = 0;
        float Cx = 0.0f, Cy = 0.0f, Cz = 0.0f, CR = 0.0f, hx = 0.0f, hy = 0.0f, hz = 0.0f;
        pg.at_step(st, [&](auto K) __attribute__((always_inline)) {
            const StepRec S = pg.step(K);
            if (RANGED) {
                ibase = st + S.blk_first;      // number of the step's environment part
                if (ibase >= test_to) return 0;
            }
            pose_step(pg, S, Tm, q, work, &sc);
            cnt = S.sph_count;
            if (cnt == 0) return 0;
            work.add(flop::kFk, flop::kPlace);
            frame_point(Tm, S.coarse[0], S.coarse[1], S.coarse[2], Cx, Cy, Cz);
            CR = S.coarse[3];
            const bool kept = S.slot >= 0, halves = kept && sc.half_off >= 0;
            if (kept) sc.put(S.slot, Cx, Cy, Cz);
            // the step's capsule half-vector (world), for its own self blocks and, kept per
            // lane, for the blocks of later steps
            if (halves || S.blk_count > 0) {
                frame_rotate(Tm, S.cap_h[0], S.cap_h[1], S.cap_h[2], hx, hy, hz);
                work.add(flop::kSelf, flop::kPlaceHalf);
                if (halves) sc.put_h(S.slot, hx, hy, hz);
            }
            return 0;
        });
        if (RANGED && ibase >= test_to) break;
        if (cnt == 0) continue;
        const bool env_part = !RANGED || ibase >= test_from;
        // the step's fine spheres, placed on first use (uniform decision)
        float cx[kSpl], cy[kSpl], cz[kSpl], cr[kSpl];
        bool placed = false;
#define VK_PLACE()                                                                  \
    if (!placed) {                                                                  \
        pg.at_step(st, [&](auto K) __attribute__((always_inline)) {                 \
            place_step(pg, pg.step(K), Tm, cx, cy, cz, cr);                         \
            return 0;                                                               \
        });                                                                         \
        work.add(flop::kFk, flop::kPlace * cnt);                                    \
        placed = true;                                                              \
    }

        if (env_part) {
            // environment: voxel broadphase per lane (candidates sorted by a lower bound of their
            // distance to the cell; stop at the first bound >= CR), then the exact link-sphere
            // test (mid-phase) and the link's fine spheres
            if (CR <= ed.vcap) {
                int b, e;
                work.add(flop::kCull, 6);
                voxel_range(ev, ed, Cx, Cy, Cz, CR, b, e);
                if (!live) e = b;
                if (wave_ballot(b < e)) {
                    VK_PLACE()
                    for (int p = b; p < e; ++p) {
                        const int2 ent = ed.vlist[p];
                        if (__int_as_float(ent.y) >= CR) break;
                        const int t = ent.x >> 28, i = ent.x & 0x0fffffff;
                        work.add(flop::kCull, flop::kBox);
                        if (hit_any(ev, t, i, Cx, Cy, Cz, CR)) {
                            work.add(flop::kFine, flop::kBox * cnt);
    #pragma unroll
                            for (int k = 0; k < kSpl; ++k)
                                if (k < cnt) col |= hit_any(ev, t, i, cx[k], cy[k], cz[k], cr[k]);
                        }
                    }
                    if (EDGE) {
                        if (wave_ballot(col)) return true;
                    } else {
                        live = !col;
                        if (!wave_ballot(live)) return col;
                    }
                }
            } else {
                // a link bounding sphere larger than the voxel lists cover: every primitive
                VK_PLACE()
                for (int i = 0; i < ev.n_sph; ++i) {
                    const float4 o = ev.rec[ev.off_sph + i];
                    VK_GATE(flop::kSphere, hit_sphere(Cx, Cy, Cz, CR, o),
                            hit_sphere(cx[k], cy[k], cz[k], cr[k], o))
                }
                for (int i = 0; i < ev.n_cap; ++i) {
                    const float4 A = ev.rec[ev.off_cap + 2 * i], B = ev.rec[ev.off_cap + 2 * i + 1];
                    VK_GATE(flop::kCapsule, hit_capsule(Cx, Cy, Cz, CR, A, B),
                            hit_capsule(cx[k], cy[k], cz[k], cr[k], A, B))
                }
                for (int i = 0; i < ev.n_cyl; ++i) {
                    const float4 A = ev.rec[ev.off_cyl + 2 * i], B = ev.rec[ev.off_cyl + 2 * i + 1];
                    VK_GATE(flop::kCylinder, hit_cylinder(Cx, Cy, Cz, CR, A, B),
                            hit_cylinder(cx[k], cy[k], cz[k], cr[k], A, B))
                }
                for (int i = 0; i < ev.n_box; ++i) {
                    const float4 X = ev.rec[ev.off_box + 4 * i], Y = ev.rec[ev.off_box + 4 * i + 1],
                                 Z = ev.rec[ev.off_box + 4 * i + 2], O = ev.rec[ev.off_box + 4 * i + 3];
                    VK_GATE(flop::kBox, hit_box(Cx, Cy, Cz, CR, X, Y, Z, O),
                            hit_box(cx[k], cy[k], cz[k], cr[k], X, Y, Z, O))
                }
            }
            // points: the clearance field rules out a link (its bounding sphere) or a sphere whose
            // neighbourhood holds no point within its radius before the grid is scanned
            if (ed.n_cells > 0) {
                const GridDev G = ld(ed.grid, 0);
                const bool near = live && !col && point_clearance(G, Cx, Cy, Cz) < CR;
                work.add(flop::kCull, flop::kClearance);
                if (wave_ballot(near)) {
                    VK_PLACE()
    #pragma unroll
                    for (int k = 0; k < kSpl; ++k) {
                        const bool scan = k < cnt && near && !col &&
                                          point_clearance(G, cx[k], cy[k], cz[k]) < cr[k];
                        if (!EDGE) {
                            // independent states: the spheres that must scan, one at a time,
                            // each by the whole wave
                            const int lane = threadIdx.x & (kWave - 1);
                            for (unsigned long long m = wave_ballot(scan); m; m &= m - 1) {
                                const int l = __builtin_ctzll(m);
                                if (grid_hit_wave(ev, G, lane_value(cx[k], l), lane_value(cy[k], l),
                                                  lane_value(cz[k], l), lane_value(cr[k], l)))
                                    col |= lane == l;
                            }
                        } else if (scan) {
                            // the lanes of an edge hold neighbouring states whose spheres
                            // mostly scan together: each lane scans its own
                            col |= grid_hit(ev, G, cx[k], cy[k], cz[k], cr[k]);
                        }
                    }
                    if (EDGE) {
                        if (wave_ballot(col)) return true;
                    } else {
                        live = !col;
                        if (!wave_ballot(live)) return col;
                    }
                }
            }

        }

        // self pairs completed by this step: gate each block with the earlier step's link
        // bounding sphere (cached centre) and then with the two links' bounding capsules (the
        // earlier one cached), then pose its link into Ta, gate each of its spheres
        // with this step's bounding sphere, and test the pairs of those that pass.  The pair
        // test runs relative to this step's bound centre C: with u_k = c_k - C and t' = t - C,
        //   |t' - u_k| < r_t + r_k  <=>  t'.u_k + al_k + r_t r_k > (|t'|^2 - r_t^2) / 2,
        //   al_k = (r_k^2 - |u_k|^2) / 2,
        // so a pair costs three FMAs, an add and a max; r_t r_k comes with the entry (-inf for
        // pairs not in its mask).  |t'| and |u_k| are at most a few link lengths, so the rounding
        // of the expanded form stays near 1e-7 m^2.
        // returns 0 to go on, 1 when the walk ends with `true` (an edge collides), 2 when it
        // ends with `col` (every state of the wave decided)
        const auto self_part = [&](auto K) __attribute__((always_inline)) {
            const StepRec S = pg.step(K);
            bool rel = false;
            float al[kSpl];
            int end = 0;
            const auto block = [&](int b) __attribute__((always_inline)) {
                const BlockRec B = pg.block(S.blk_first + b);
                float ax, ay, az;
                sc.get(B.slot_a, ax, ay, az);
                const float dx = ax - Cx, dy = ay - Cy, dz = az - Cz;
                const float rr = B.ra + CR;
                work.add(flop::kSelf, flop::kPair);
                if (!wave_ballot(live && fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rr * rr)) return false;
                // second gate, still without posing A: the segments c -+ h of the two links'
                // bounding capsules (A's half-vector from the cache, in half precision, whose
                // error A's cap_rq covers); without the halves in the cache, A's bounding sphere
                // against this step's capsule
                if (sc.half_off < 0) {
                    const float px = Cx - hx, py = Cy - hy, pz = Cz - hz;
                    const float rx = ax - px, ry = ay - py, rz = az - pz;
                    const float t = fminf(fmaxf(2.0f * fmaf(rx, hx, fmaf(ry, hy, rz * hz)) * S.cap_inv,
                                                0.0f), 1.0f);
                    const float ex = fmaf(-2.0f * t, hx, rx), ey = fmaf(-2.0f * t, hy, ry),
                                ez = fmaf(-2.0f * t, hz, rz);
                    const float rc = B.ra + S.cap_r;
                    work.add(flop::kSelf, flop::kSphereCapsule);
                    if (!wave_ballot(live && fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rc * rc))
                        return false;
                } else {
                    float hax, hay, haz;
                    sc.get_h(B.slot_a, hax, hay, haz);
                    const float a = 4.0f * fmaf(hax, hax, fmaf(hay, hay, haz * haz));
                    const float ia = a > 0.0f ? __builtin_amdgcn_rcpf(a) : 0.0f;
                    const float d2 = seg_seg2(ax - hax, ay - hay, az - haz, 2.0f * hax, 2.0f * hay,
                                              2.0f * haz, a, ia, Cx - hx, Cy - hy, Cz - hz, 2.0f * hx,
                                              2.0f * hy, 2.0f * hz, S.cap_uu, S.cap_inv);
                    const float rc = B.rqa + S.cap_r;
                    work.add(flop::kSelf, flop::kCapsuleCapsule);
                    if (!wave_ballot(live && d2 < rc * rc)) return false;
                }
                pose_block(pg, B, Ta, ta_link, ta_depth, sc, q, work);
                const float ox = Ta.p[0] - Cx, oy = Ta.p[1] - Cy, oz = Ta.p[2] - Cz;
                float D = -__builtin_inff();
                for (int e = 0; e < B.ent_count; ++e) {
                    const EntryRec E = pg.entry(B.ent_first + e);
                    const float tx = fmaf(Ta.r[0], E.x, fmaf(Ta.r[1], E.y, fmaf(Ta.r[2], E.z, ox)));
                    const float ty = fmaf(Ta.r[3], E.x, fmaf(Ta.r[4], E.y, fmaf(Ta.r[5], E.z, oy)));
                    const float tz = fmaf(Ta.r[6], E.x, fmaf(Ta.r[7], E.y, fmaf(Ta.r[8], E.z, oz)));
                    const float t2 = fmaf(tx, tx, fmaf(ty, ty, tz * tz));
                    work.add(flop::kRepose, flop::kPlace);
                    work.add(flop::kSelf, flop::kPair);
                    if (!wave_ballot(live && t2 < E.gate2)) continue;
                    if (!rel) {                      // this step's spheres, relative to C
                        if (!placed) {
                            place_step(pg, S, Tm, cx, cy, cz, cr);
                            work.add(flop::kFk, flop::kPlace * cnt);
                            placed = true;
                        }
#pragma unroll
                        for (int k = 0; k < kSpl; ++k) {
                            cx[k] -= Cx;
                            cy[k] -= Cy;
                            cz[k] -= Cz;
                            al[k] = fmaf(-0.5f, fmaf(cx[k], cx[k], fmaf(cy[k], cy[k], cz[k] * cz[k])),
                                         0.5f * cr[k] * cr[k]);
                        }
                        rel = true;
                    }
                    // every slot: unpaired and unused ones carry rr = -inf
                    float M = -__builtin_inff();
#pragma unroll
                    for (int k = 0; k < kSpl; ++k)
                        M = fmaxf(M, fmaf(tx, cx[k], fmaf(ty, cy[k], fmaf(tz, cz[k], al[k]))) + E.rr[k]);
                    work.add(flop::kSelf, flop::kPair * __builtin_popcount(E.mask));
                    D = fmaxf(D, M - fmaf(0.5f, t2, E.nhr2));
                }
                col |= D > 0.0f;
                if (EDGE) {
                    if (wave_ballot(col)) {
                        end = 1;
                        return true;
                    }
                } else {
                    live = !col;
                    if (!wave_ballot(live)) {
                        end = 2;
                        return true;
                    }
                }
                return false;
            };
            int b_lo = 0, b_hi = S.blk_count;
            if (RANGED) {                      // the blocks inside [test_from, test_to)
                b_lo = max(0, test_from - ibase - 1);
                b_hi = min(S.blk_count, test_to - ibase - 1);
            }
            for (int b = b_lo; b < b_hi; ++b)
                if (block(b)) break;
            return end;
        };
        // one copy of the self part runs on the step's records at run time (compiling it per
        // step, with the blocks and entries unrolled, made the specialised kernel spill hundreds
        // of registers and outgrow the instruction cache)
        const int ended = self_part(st);
        if (EDGE && ended == 1) return true;
        if (!EDGE && ended == 2) return col;
#undef VK_PLACE
    }
    return EDGE ? false : col;
}


// ---------------------------------------------------------------------------------------------
// Edge validation.  One wave validates one edge: states in rake order, first hit ends it.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int edge_count(const float *a, const float *b, int dof, float res) {
    // n = max(2, ceil(L / res) + 1), L = max_j |b_j - a_j| in double: the difference of two
    // floats is exact in double, so this matches a double-precision evaluation bit for bit.
    double L = 0.0;
    for (int j = 0; j < dof; ++j) L = fmax(L, fabs((double)ld(b, j) - (double)ld(a, j)));
    const double n = ceil(L / (double)res) + 1.0;
    return n < 2.0 ? 2 : (n > 2147483647.0 ? 2147483647 : (int)n);
}

// Endpoints of edge e.  Returns 0 for an edge to validate, 1 for a hole (an index pair with a
// negative entry: no edge, flag 0) and 2 for an index past the node array (flag 1).
__device__ __forceinline__ int edge_ends(const EdgeSrc &src, int dof, int64_t e, const float *&a,
                                         const float *&b) {
    if (!src.pairs) {
        a = src.qa + e * dof;
        b = src.qb + e * dof;
        return 0;
    }
    const int64_t i = ld(src.pairs, 2 * e), j = ld(src.pairs, 2 * e + 1);
    if (i < 0 || j < 0) return 1;
    if (i >= src.n_nodes || j >= src.n_nodes) return 2;
    a = src.qa + i * dof;
    b = src.qa + j * dof;
    return 0;
}

// Has another part of the edge already found a collision (its flag set)?  A coherent load:
// the flag may have been stored by a wave on another compute unit.
__device__ __forceinline__ bool edge_flagged(const uint8_t *flag) {
    return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Part `part` of `parts` of the edge's rake: the rake steps k = part, part + parts, ... (all of
// them for parts == 1).  Every part starts with a step that samples the whole motion, and a
// part stops early once another part has flagged the edge (flag, read only when parts > 1).
// With RANGED only the walk's tests [test_from, test_to) run in each state.
template <bool RANGED = false, class P, class V, class W = NoWork>
__device__ __forceinline__ uint8_t edge_body(const P &pg, const V &ev, const EnvDev &ed,
                                             const StepCache &sc, const float *a, const float *b,
                                             int n, W &&work = W(), int part = 0, int parts = 1,
                                             const uint8_t *flag = nullptr, int test_from = 0,
                                             int test_to = kAllTests) {
    bool bad = false;
    for (int j = 0; j < pg.dof(); ++j) bad |= !isfinite(ld(a, j)) || !isfinite(ld(b, j));
    if (bad) return 1;
    if (n < 2) n = 2;
    if (n > kMaxEdgeStates) return 1;         // too long to validate: reported as colliding
    const int lane = threadIdx.x & (kWave - 1);
    const int stride = (n + kWave - 1) / kWave;
    const float inv = 1.0f / (float)(n - 1);
    for (int k = part; k < stride; k += parts) {
        if (parts > 1 && k != part && edge_flagged(flag)) return 0;
        int idx = lane * stride + k;
        work.rake_slot(idx < n);
        idx = idx < n ? idx : n - 1;          // surplus lanes repeat the last state
        const float t = idx == n - 1 ? 1.0f : (float)idx * inv;
        QEdge qs{a, b, t};
        if (walk_collide<true, RANGED>(pg, ev, ed, qs, sc, false, test_from, test_to, work))
            return 1;
    }
    return 0;
}

// Ticket from a counter with no lane-dependent branch: every lane executes the atomic, lane 0
// adds 1 and the others add 0, so lane 0's returned value is the wave's ticket, broadcast from
// the first active lane (lane 0; the whole wave is active here).  Keeping lane-dependent control
// flow out of the persistent loop matters: a lane-0-only `if` around the atomic can be threaded
// by the compiler across iterations, after which the broadcast reads a lane that never took a
// ticket.

__device__ __forceinline__ unsigned long long take_ticket(unsigned long long *ctr, int lane) {
    return uniform_u64(atomicAdd(ctr, lane == 0 ? 1ull : 0ull));
}

// Persistent work distribution.  The items [0, n) are split into kQueues equal parts; part p is
// handed out in chunks of `chunk` items by the counter at queue[p * kQueueWords].  A wave starts
// at part (workgroup index mod kQueues) -- consecutive workgroups are placed on different XCDs,
// so the waves of one XCD mostly share a counter and no counter serialises the whole chip -- and
// moves to the next part once its part is drained.  A part visited after the home part is first
// read with a plain atomic load, so drained parts cost no read-modify-write.  A wave leaves each
// part at most once, so the loop ends after at most kQueues drained parts.
struct Puller {
    unsigned long long *queue;
    int64_t n;
    int chunk, part, left;
};

__device__ __forceinline__ Puller make_puller(unsigned long long *queue, int64_t n, int chunk) {
    return Puller{queue, n, chunk, (int)(blockIdx.x % kQueues), kQueues};
}

__device__ __forceinline__ bool pull(Puller &p, int lane, int64_t &first, int64_t &count) {
    while (p.left > 0) {
        const int64_t lo = p.n * p.part / kQueues, hi = p.n * (p.part + 1) / kQueues;
        unsigned long long *ctr = p.queue + (size_t)p.part * kQueueWords;
        bool open = true;
        if (p.left < kQueues) {
            const unsigned long long seen =
                uniform_u64(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            open = (int64_t)seen * p.chunk < hi - lo;
        }
        if (open) {
            const int64_t f = (int64_t)take_ticket(ctr, lane) * p.chunk;
            if (f < hi - lo) {
                first = lo + f;
                count = hi - lo - f < p.chunk ? hi - lo - f : p.chunk;
                return true;
            }
        }
        p.part = p.part + 1 == kQueues ? 0 : p.part + 1;
        --p.left;
    }
    return false;
}


// The persistent edge launch: waves pull chunks of work items from the work queue and walk
// each with the rake (the kernels of both program sources call this).  With one part per edge
// an item is an edge and its flag is stored as found.  An edge can also be split over
// parts x tparts waves: `parts` split its rake steps (long edges) and `tparts` split the walk's
// tests into that many ranges of about equal count (small batches, whose launch is bound by
// the latency of one walk).  Item i is then part p = i / n_edges of edge i % n_edges (part-major,
// so the parts of one edge sit in different queue ranges and run on different waves at about
// the same time), with rake part p % parts and test range p / parts; the flags were zeroed and
// a part stores 1 when it finds a collision.
// MULTI = false compiles the one-wave form (parts and tparts are then taken as 1), which keeps
// the multi-part bookkeeping out of the register allocation of the common case.
template <int STAGE, bool COUNT, bool MULTI, class P>
__device__ __forceinline__ void validate_edges_body(const P &pg, const EnvDev &ed,
                                                    const float4 *__restrict__ env_rec,
                                                    const EdgeSrc &src, int64_t n_edges, float res,
                                                    uint8_t *__restrict__ out,
                                                    unsigned long long *__restrict__ queue, int chunk,
                                                    unsigned long long *__restrict__ flops, int cf,
                                                    int parts_in, int tparts_in) {
    const int parts = MULTI ? parts_in : 1;
    const int tparts = MULTI ? tparts_in : 1;
    const RobotDev &rb = pg.rb;
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const int lane = threadIdx.x & (kWave - 1);
    typename std::conditional<COUNT, Work, NoWork>::type work;
    Puller pl = make_puller(queue, n_edges * parts * tparts, chunk);
    int64_t first, count;
    while (pull(pl, lane, first, count)) {
        for (int64_t item = first; item < first + count; ++item) {
            const int p = MULTI ? (int)(item / n_edges) : 0;
            const int64_t e = MULTI ? item - p * n_edges : item;
            const int part = MULTI ? p % parts : 0;
            int t0 = 0, t1 = kAllTests;
            if (MULTI && tparts > 1) {
                const int y = p / parts;
                t0 = (int)((int64_t)y * rb.n_tests / tparts);
                t1 = (int)((int64_t)(y + 1) * rb.n_tests / tparts);
            }
            const float *a = nullptr, *b = nullptr;
            const int kind = edge_ends(src, pg.dof(), e, a, b);
            uint8_t hit = kind == 2 ? 1 : 0;
            if (kind == 0) {
                const int n = src.nst ? ld(src.nst, e) : edge_count(a, b, pg.dof(), res);
                hit = MULTI ? edge_body<MULTI>(pg, ev, ed, sc, a, b, n, work, part, parts, out + e,
                                               t0, t1)
                            : edge_body(pg, ev, ed, sc, a, b, n, work);
            }
            if (!MULTI)
                out[e] = hit;                 // wave-uniform value, same address in every lane
            else if (hit)
                out[e] = 1;
        }
    }
    if constexpr (COUNT) {
        // flops[0] the total, flops[1..6] the categories, flops[7] the rake slots of real states
        unsigned long long v[flop::kCats + 1];
#pragma unroll
        for (int c = 0; c < flop::kCats; ++c) v[c] = work.f[c];
        v[flop::kCats] = work.visits;
#pragma unroll
        for (int c = 0; c <= flop::kCats; ++c)
            for (int m = 1; m < kWave; m <<= 1) v[c] += __shfl_xor(v[c], m);
        unsigned long long total = 0;
#pragma unroll
        for (int c = 0; c < flop::kCats; ++c) total += v[c];
        atomicAdd(flops + 0, lane == 0 ? total : 0ull);
#pragma unroll
        for (int c = 0; c <= flop::kCats; ++c) atomicAdd(flops + 1 + c, lane == 0 ? v[c] : 0ull);
    }
}

}  // namespace vk
