// HIP kernels for gfx950: sphere FK, state validation, rake-ordered edge validation (persistent
// work queue and one-launch-per-edge), and the squared-penetration cost with its adjoint.
//
// Mapping (Sec. III-A..D of the paper, re-designed for 64-wide CDNA wavefronts):
//   * one lane = one configuration; a wavefront is the "vector" of configurations;
//   * configurations are SoA in HBM, so lane i's load of joint j is one coalesced access;
//   * the robot program (link steps, self-pair blocks) and the environment are wave-uniform:
//     the robot through scalar loads, the environment staged once per workgroup in LDS;
//   * per link: pose it, place its spheres, test them against the environment behind the
//     link's bounding sphere (mid-phase, Sec. III-D), then test the self pairs it completes --
//     checks are interleaved into FK and the walk stops at the first hit (Sec. III-D);
//   * edges use the rake: lane l takes state l*ceil(n/64) + k at step k, so the first step
//     samples the whole motion (Sec. III-D, Fig. 2) and a wave ballot ends the edge early.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "vk_launch.hpp"
#include "vk_walk.hpp"

namespace vk {

// ---------------------------------------------------------------------------------------------
// fk_spheres: one lane per state; writes [S][3][ldc] with streaming (non-temporal) stores: the
// centres are not read back by this library, and keeping them out of the caches lets the write
// stream run at 5.4-5.5 TB/s instead of 4.6-4.7.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fk_spheres(RobotDev rb, const float *__restrict__ q,
                                                    int64_t n, int64_t ldq,
                                                    float *__restrict__ out, int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    QState qs{q, ldq, active ? i : 0};
    Frame T;
    frame_identity(T);
    for (int st = 0; st < rb.n_steps; ++st) {
        const StepRec S = ld(rb.steps, st);
        pose_step(DynProg{rb}, S, T, qs);
        for (int k = 0; k < S.sph_count; ++k) {
            const int s = S.sph_first + k;
            const float4 l = ld(rb.spheres, s);
            float x, y, z;
            frame_point(T, l.x, l.y, l.z, x, y, z);
            if (active) {
                __builtin_nontemporal_store(x, &out[(3 * (int64_t)s + 0) * ldc + i]);
                __builtin_nontemporal_store(y, &out[(3 * (int64_t)s + 1) * ldc + i]);
                __builtin_nontemporal_store(z, &out[(3 * (int64_t)s + 2) * ldc + i]);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// validate_states: one lane per state.
// ---------------------------------------------------------------------------------------------
// With one range the whole walk runs and every flag is stored.  A small batch (too few waves to
// fill the chip) is split into ranges of the walk's tests (each step's environment part and
// each of its self blocks, numbered in walk order): block row y runs tests [b[y], b[y + 1])
// only, posing the earlier steps; the flags were zeroed and a range stores 1 where it finds a
// collision, so a state's flag is the OR over the ranges, the flag of the whole walk.
// four waves per SIMD (at most 128 VGPRs): left alone the compiler takes 133 and fits three
template <int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_validate_states(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                      const float *__restrict__ q, int64_t n, int64_t ldq,
                      uint8_t *__restrict__ out, int cf, StepRanges ranges) {
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    QState qs{q, ldq, active ? i : 0};
    bool col = !active;                       // inactive lanes count as decided
    if (active)
        for (int j = 0; j < rb.dof; ++j) col |= !isfinite(qs(j));
    if (ranges.n <= 1) {
        col = walk_collide<false>(DynProg{rb}, ev, ed, qs, sc, col, 0, kAllTests);
        if (active) out[i] = col ? 1 : 0;
        return;
    }
    const int y = blockIdx.y;
    col = walk_collide<false>(DynProg{rb}, ev, ed, qs, sc, col, ranges.b[y], ranges.b[y + 1]);
    if (active && col) out[i] = 1;
}

// Two-pass state validation.  In a wave of independent states the walk lasts until its last
// live lane ends, so when most states collide early a few free lanes keep whole waves walking
// at low occupancy of their lanes.  Pass 1 runs the walk's tests before number `split` (the
// first test of a link step; tests are numbered as for the ranges above) on every state and
// appends the states still free to a survivor list (one atomic per wave); pass 2 walks the
// survivors packed densely into waves, posing the earlier steps again and running the rest.
// Flags are those of the single pass.
// four waves per SIMD: without the bound the compiler takes 131 VGPRs, three waves; at 128 it
// spills one or two and the point-cloud batch runs 2.5 % faster
template <int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_validate_states_screen(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                             const float *__restrict__ q, int64_t n, int64_t ldq,
                             uint8_t *__restrict__ out, int cf, int split,
                             int32_t *__restrict__ surv, unsigned long long *__restrict__ n_surv) {
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    QState qs{q, ldq, active ? i : 0};
    bool col = !active;
    if (active)
        for (int j = 0; j < rb.dof; ++j) col |= !isfinite(qs(j));
    col = walk_collide<false>(DynProg{rb}, ev, ed, qs, sc, col, 0, split);
    const bool keep = active && !col;
    if (active && col) out[i] = 1;
    const unsigned long long m = wave_ballot(keep);
    const unsigned long long base =
        uniform_u64(atomicAdd(n_surv, lane == 0 ? (unsigned long long)__popcll(m) : 0ull));
    const int below = __builtin_amdgcn_mbcnt_hi((unsigned int)(m >> 32),
                                                __builtin_amdgcn_mbcnt_lo((unsigned int)m, 0u));
    if (keep) surv[base + below] = (int32_t)i;
}

template <int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_validate_states_rest(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                           const float *__restrict__ q, int64_t ldq, uint8_t *__restrict__ out,
                           int cf, int split, const int32_t *__restrict__ surv,
                           const unsigned long long *__restrict__ n_surv) {
    const int64_t count = (int64_t)*n_surv;
    if ((int64_t)blockIdx.x * blockDim.x >= count) return;     // whole workgroup past the list
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = g < count;
    const int64_t i = active ? surv[g] : 0;
    QState qs{q, ldq, i};
    bool col = !active;
    col = walk_collide<false>(DynProg{rb}, ev, ed, qs, sc, col, split, kAllTests);
    if (active) out[i] = col ? 1 : 0;
}

// Waves per SIMD the persistent edge kernel is compiled for (register budget 512 / waves).
#ifndef VK_EDGE_WAVES
#define VK_EDGE_WAVES 4
#endif

template <int STAGE, bool COUNT, bool MULTI>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(VK_EDGE_WAVES, 8)))
    k_validate_edges(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                     EdgeSrc src, int64_t n_edges, float res,
                     uint8_t *__restrict__ out, unsigned long long *__restrict__ queue,
                     int chunk, unsigned long long *__restrict__ flops, int cf, int parts,
                     int tparts) {
    validate_edges_body<STAGE, COUNT, MULTI>(DynProg{rb}, ed, env_rec, src, n_edges, res, out,
                                             queue, chunk, flops, cf, parts, tparts);
}

template <int STAGE>
__global__ void __launch_bounds__(64)
    k_validate_edge_one(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                        EdgeSrc src, int64_t e, float res, uint8_t *__restrict__ out, int cf) {
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const float *a = nullptr, *b = nullptr;
    const int kind = edge_ends(src, rb.dof, e, a, b);
    uint8_t hit = kind == 2 ? 1 : 0;
    if (kind == 0) {
        const int n = src.nst ? ld(src.nst, e) : edge_count(a, b, rb.dof, res);
        hit = edge_body(DynProg{rb}, ev, ed, sc, a, b, n);
    }
    out[e] = hit;                             // wave-uniform value
}

// Mixed-robot batch: every edge set has its own robot and environment; one persistent launch
// pulls edges from a single queue across all sets.  The environment is read from global
// memory with wave-uniform loads (it changes from item to item, so it is not staged in LDS).
// edge_set[e] names edge e's set, so finding it costs one load.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(VK_EDGE_WAVES, 8)))
    k_validate_edge_batch(const BatchSet *__restrict__ sets, const int32_t *__restrict__ edge_set,
                          int n_sets, int64_t total, float res, const float *__restrict__ qa,
                          const float *__restrict__ qb, uint8_t *__restrict__ out,
                          unsigned long long *__restrict__ queue, int chunk, int cache_floats, int cf) {
    extern __shared__ float4 lds_dyn[];
    float *cache_base = reinterpret_cast<float *>(lds_dyn) + (threadIdx.x / kWave) * cache_floats;
    const int lane = threadIdx.x & (kWave - 1);
    Puller pl = make_puller(queue, total, chunk);
    int64_t first, count;
    while (pull(pl, lane, first, count))
    for (int64_t e = first; e < first + count; ++e) {
        const BatchSet S = ld(sets, ld(edge_set, e));
        const int64_t local = e - S.first;
        const float *a = qa + S.qa_offset + local * S.rb.dof;
        const float *b = qb + S.qa_offset + local * S.rb.dof;
        const int n = edge_count(a, b, S.rb.dof, res);
        const EnvView ev = make_view<0>(S.env, nullptr);
        const StepCache sc = make_step_cache(cache_base, S.rb.n_slots, cf);
        const uint8_t hit = edge_body(DynProg{S.rb}, ev, S.env, sc, a, b, n);
        out[S.out_offset + local] = hit;      // wave-uniform value
    }
}

__global__ void k_zero_u8(uint8_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int n, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[(size_t)i * stride] = v;
}

// The queue counters and a batch's flags zeroed by one launch (edges split over several waves
// store only the 1s).
__global__ void k_reset_queue_flags(unsigned long long *queue, uint8_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kQueues) queue[i * kQueueWords] = 0ull;
    if (i < n) out[i] = 0;
}

// ---------------------------------------------------------------------------------------------
// Squared-penetration cost.  Every pair contributes max(0, -clearance)^2; the per-step
// bounding sphere still gates the fine tests (no penetration of the bound implies none of the
// fine spheres), but there is no early exit.
// ---------------------------------------------------------------------------------------------
template <bool GRAD>
struct CostAcc;

// Penetration of sphere k against a primitive with signed distance sd and gradient g;
// accumulates the cost and (GRAD) the force d cost / d c = -2 p g.
#define VK_PEN(SDEXPR)                                                                \
    {                                                                                 \
        float gx, gy, gz;                                                             \
        const float sd = (SDEXPR);                                                    \
        const float p = cr[k] - sd;                                                   \
        if (p > 0.0f) {                                                               \
            cost = fmaf(p, p, cost);                                                  \
            if (GRAD) {                                                               \
                fx[k] = fmaf(-2.0f * p, gx, fx[k]);                                   \
                fy[k] = fmaf(-2.0f * p, gy, fy[k]);                                   \
                fz[k] = fmaf(-2.0f * p, gz, fz[k]);                                   \
            }                                                                         \
        }                                                                             \
    }

#define VK_COST_GATE(COARSE, SDEXPR)                                                  \
    if (wave_ballot(live && (COARSE))) {                                              \
        _Pragma("unroll") for (int k = 0; k < kSpl; ++k) if (k < cnt) VK_PEN(SDEXPR) \
    }

// Per-link force/moment slots (in LDS or in global scratch): slot (link, component) for each
// lane of the wave.
struct LinkSlots {
    float *base;               // [n_links][6][64] for this wave
    int lane;
    __device__ __forceinline__ float &at(int link, int c) const {
        return base[(link * 6 + c) * kWave + lane];
    }
    // a link's six values, read and written as a group
    __device__ __forceinline__ void load6(int link, float (&v)[6]) const {
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = at(link, c);
    }
    __device__ __forceinline__ void store6(int link, const float (&v)[6]) const {
#pragma unroll
        for (int c = 0; c < 6; ++c) at(link, c) = v[c];
    }
    // a force and its moment about the world origin, summed in registers by the caller over
    // the spheres of one step or the entries of one self block: one update of the link's slots
    __device__ __forceinline__ void add_fm(int link, float fx, float fy, float fz, float mx,
                                           float my, float mz) const {
        at(link, 0) += fx;
        at(link, 1) += fy;
        at(link, 2) += fz;
        at(link, 3) += mx;
        at(link, 4) += my;
        at(link, 5) += mz;
    }
};

// Running force and moment (about the world origin, p x f) of forces f applied at points p.
struct ForceSum {
    float fx = 0.0f, fy = 0.0f, fz = 0.0f, mx = 0.0f, my = 0.0f, mz = 0.0f;
    __device__ __forceinline__ void add(float px, float py, float pz, float gx, float gy, float gz) {
        fx += gx;
        fy += gy;
        fz += gz;
        mx = fmaf(py, gz, mx) - pz * gy;
        my = fmaf(pz, gx, my) - px * gz;
        mz = fmaf(px, gy, mz) - py * gx;
    }
    __device__ __forceinline__ void to(const LinkSlots &s, int link) const {
        s.add_fm(link, fx, fy, fz, mx, my, mz);
    }
};

template <bool GRAD, class Q>
__device__ float cost_walk(const RobotDev &rb, const EnvView &ev, const EnvDev &ed, const Q &q,
                           const StepCache &sc, bool live, const LinkSlots &slots) {
    Frame Tm, Ta;
    frame_identity(Tm);
    frame_identity(Ta);
    int ta_link = 0, ta_depth = 0;
    float cost = 0.0f;
    for (int st = 0; st < rb.n_steps; ++st) {
        const StepRec S = ld(rb.steps, st);
        pose_step(DynProg{rb}, S, Tm, q, NoWork(), &sc);
        const int cnt = S.sph_count;
        if (cnt == 0) continue;
        float cx[kSpl], cy[kSpl], cz[kSpl], cr[kSpl], fx[kSpl], fy[kSpl], fz[kSpl];
#pragma unroll
        for (int k = 0; k < kSpl; ++k) {
            cx[k] = cy[k] = cz[k] = cr[k] = 0.0f;
            fx[k] = fy[k] = fz[k] = 0.0f;
            if (k < cnt) {
                const float4 s = ld(rb.spheres, S.sph_first + k);
                frame_point(Tm, s.x, s.y, s.z, cx[k], cy[k], cz[k]);
                cr[k] = s.w;
            }
        }
        float Cx, Cy, Cz;
        frame_point(Tm, S.coarse[0], S.coarse[1], S.coarse[2], Cx, Cy, Cz);
        const float CR = S.coarse[3];
        const bool halves = S.slot >= 0 && sc.half_off >= 0;
        if (S.slot >= 0) sc.put(S.slot, Cx, Cy, Cz);
        float hx = 0.0f, hy = 0.0f, hz = 0.0f;      // capsule half-vector (world), as in the walk
        if (halves || S.blk_count > 0) {
            frame_rotate(Tm, S.cap_h[0], S.cap_h[1], S.cap_h[2], hx, hy, hz);
            if (halves) sc.put_h(S.slot, hx, hy, hz);
        }
        if (CR <= ed.vcap) {
            int b, e;
            voxel_range(ev, ed, Cx, Cy, Cz, CR, b, e);
            if (!live) e = b;
            for (int p = b; p < e; ++p) {
                const int2 ent = ed.vlist[p];
                if (__int_as_float(ent.y) >= CR) break;
                const int t = ent.x >> 28, i = ent.x & 0x0fffffff;
                if (!hit_any(ev, t, i, Cx, Cy, Cz, CR)) continue;
#pragma unroll
                for (int k = 0; k < kSpl; ++k)
                    if (k < cnt) VK_PEN(sd_any(ev, t, i, cx[k], cy[k], cz[k], gx, gy, gz))
            }
        } else {
            for (int i = 0; i < ev.n_sph; ++i) {
                const float4 o = ev.rec[ev.off_sph + i];
                VK_COST_GATE(hit_sphere(Cx, Cy, Cz, CR, o), sd_sphere(cx[k], cy[k], cz[k], o, gx, gy, gz))
            }
            for (int i = 0; i < ev.n_cap; ++i) {
                const float4 A = ev.rec[ev.off_cap + 2 * i], B = ev.rec[ev.off_cap + 2 * i + 1];
                VK_COST_GATE(hit_capsule(Cx, Cy, Cz, CR, A, B),
                             sd_capsule(cx[k], cy[k], cz[k], A, B, gx, gy, gz))
            }
            for (int i = 0; i < ev.n_cyl; ++i) {
                const float4 A = ev.rec[ev.off_cyl + 2 * i], B = ev.rec[ev.off_cyl + 2 * i + 1];
                VK_COST_GATE(hit_cylinder(Cx, Cy, Cz, CR, A, B),
                             sd_cylinder(cx[k], cy[k], cz[k], A, B, gx, gy, gz))
            }
            for (int i = 0; i < ev.n_box; ++i) {
                const float4 X = ev.rec[ev.off_box + 4 * i], Y = ev.rec[ev.off_box + 4 * i + 1],
                             Z = ev.rec[ev.off_box + 4 * i + 2], O = ev.rec[ev.off_box + 4 * i + 3];
                VK_COST_GATE(hit_box(Cx, Cy, Cz, CR, X, Y, Z, O),
                             sd_box(cx[k], cy[k], cz[k], X, Y, Z, O, gx, gy, gz))
            }
        }
        if (ed.n_cells > 0) {
            // the spheres whose neighbourhood may hold a point, one at a time, each by the whole
            // wave: 64 points of a row per round, the penetration sums added over the wave
            const GridDev G = ld(ed.grid, 0);
            const bool near = live && point_clearance(G, Cx, Cy, Cz) < CR;
            if (wave_ballot(near)) {
                const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
                for (int k = 0; k < kSpl; ++k) {
                    const bool scan = near && k < cnt &&
                                      point_clearance(G, cx[k], cy[k], cz[k]) < cr[k];
                    for (unsigned long long m = wave_ballot(scan); m; m &= m - 1) {
                        const int l = __builtin_ctzll(m);
                        const float sx = lane_value(cx[k], l), sy = lane_value(cy[k], l),
                                    sz = lane_value(cz[k], l), sr = lane_value(cr[k], l);
                        float c = 0.0f, ux = 0.0f, uy = 0.0f, uz = 0.0f;
                        grid_rows<true>(ev, G, sx, sy, sz, sr, [&](int b, int e) {
                            for (int p = b + lane; p - lane < e; p += kWave) {
                                if (p >= e) continue;
                                float gx, gy, gz;
                                const float pen = sr - sd_sphere(sx, sy, sz, G.pts[p], gx, gy, gz);
                                if (pen > 0.0f) {
                                    c = fmaf(pen, pen, c);
                                    if (GRAD) {
                                        ux = fmaf(-2.0f * pen, gx, ux);
                                        uy = fmaf(-2.0f * pen, gy, uy);
                                        uz = fmaf(-2.0f * pen, gz, uz);
                                    }
                                }
                            }
                            return false;
                        });
                        c = wave_sum(c);
                        if (GRAD) {
                            ux = wave_sum(ux);
                            uy = wave_sum(uy);
                            uz = wave_sum(uz);
                        }
                        if (lane == l) {
                            cost += c;
                            if (GRAD) {
                                fx[k] += ux;
                                fy[k] += uy;
                                fz[k] += uz;
                            }
                        }
                    }
                }
            }
        }
        for (int b = 0; b < S.blk_count; ++b) {
            const BlockRec B = ld(rb.blocks, S.blk_first + b);
            float ax, ay, az;
            sc.get(B.slot_a, ax, ay, az);
            const float dx = ax - Cx, dy = ay - Cy, dz = az - Cz;
            const float rr = B.ra + CR;
            if (!wave_ballot(live && fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rr * rr)) continue;
            // the gates of the collision walk: no pair they rule out can penetrate, so the
            // cost and its gradient do not change
            if (sc.half_off >= 0) {
                float hax, hay, haz;
                sc.get_h(B.slot_a, hax, hay, haz);
                const float a = 4.0f * fmaf(hax, hax, fmaf(hay, hay, haz * haz));
                const float ia = a > 0.0f ? __builtin_amdgcn_rcpf(a) : 0.0f;
                const float d2 = seg_seg2(ax - hax, ay - hay, az - haz, 2.0f * hax, 2.0f * hay,
                                          2.0f * haz, a, ia, Cx - hx, Cy - hy, Cz - hz, 2.0f * hx,
                                          2.0f * hy, 2.0f * hz, S.cap_uu, S.cap_inv);
                const float rc = B.rqa + S.cap_r;
                if (!wave_ballot(live && d2 < rc * rc)) continue;
            }
            pose_block(DynProg{rb}, B, Ta, ta_link, ta_depth, sc, q);
            ForceSum fa;                         // the forces on A's spheres from this block
            for (int e = 0; e < B.ent_count; ++e) {
                const EntryRec E = ld(rb.entries, B.ent_first + e);
                float tx, ty, tz;
                frame_point(Ta, E.x, E.y, E.z, tx, ty, tz);
                {
                    const float ex = tx - Cx, ey = ty - Cy, ez = tz - Cz;
                    if (!wave_ballot(live && fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < E.gate2)) continue;
                }
                float gtx = 0.0f, gty = 0.0f, gtz = 0.0f;
#pragma unroll
                for (int k = 0; k < kSpl; ++k) {
                    if ((E.mask >> k) & 1u) {
                        float ux, uy, uz;
                        const float d = sd_grad_point(cx[k], cy[k], cz[k], tx, ty, tz, ux, uy, uz);
                        const float p = E.r + cr[k] - d;
                        if (p > 0.0f) {
                            cost = fmaf(p, p, cost);
                            if (GRAD) {
                                const float w = -2.0f * p;
                                fx[k] = fmaf(w, ux, fx[k]);
                                fy[k] = fmaf(w, uy, fy[k]);
                                fz[k] = fmaf(w, uz, fz[k]);
                                gtx = fmaf(-w, ux, gtx);
                                gty = fmaf(-w, uy, gty);
                                gtz = fmaf(-w, uz, gtz);
                            }
                        }
                    }
                }
                if (GRAD) fa.add(tx, ty, tz, gtx, gty, gtz);
            }
            if (GRAD) {
                float pre[6];
                slots.load6(B.link, pre);
                pre[0] += fa.fx;
                pre[1] += fa.fy;
                pre[2] += fa.fz;
                pre[3] += fa.mx;
                pre[4] += fa.my;
                pre[5] += fa.mz;
                slots.store6(B.link, pre);
            }
        }
        if (GRAD) {
            ForceSum fs;                         // the forces on this step's spheres
#pragma unroll
            for (int k = 0; k < kSpl; ++k)
                if (k < cnt) fs.add(cx[k], cy[k], cz[k], fx[k], fy[k], fz[k]);
            if (S.joint >= 0) {
                // the link's first step: nothing has reached its slots since they were zeroed
                // (self blocks update only earlier links), so they are written, not updated
                const float v[6] = {fs.fx, fs.fy, fs.fz, fs.mx, fs.my, fs.mz};
                slots.store6(S.link, v);
            } else {
                fs.to(slots, S.link);
            }
        }
    }
    return cost;
}

template <int STAGE>
__global__ void __launch_bounds__(256)
    k_cost_fwd(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
               const float *__restrict__ q, int64_t n, int64_t ldq, float *__restrict__ cost, int cf) {
    extern __shared__ float4 lds_dyn[];
    float *lf = reinterpret_cast<float *>(lds_dyn);
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    QState qs{q, ldq, active ? i : 0};
    bool finite = true;
    for (int j = 0; j < rb.dof; ++j) finite &= isfinite(qs(j));
    LinkSlots none{nullptr, 0};
    const float c = cost_walk<false>(rb, ev, ed, qs, sc, active && finite, none);
    if (active) cost[i] = finite ? c : __builtin_nanf("");
}

// Backward: forces per link accumulated in LDS, suffix sums over the tree, then
// dq_j = z_j . (M_j - o_j x F_j) with (F_j, M_j) the force and moment (about the origin) of
// everything joint j moves and (z_j, o_j) the axis and origin of joint j's frame.
// The slots live in LDS ([slots of every wave of the block][walk caches][env records]) or, with
// GSLOT, in global memory (gslots: every wave's slots, in wave order), which frees the LDS that
// holds the backward kernel's occupancy down.
template <int STAGE, bool GSLOT>
__device__ __forceinline__ void cost_bwd_body(const RobotDev &rb, const EnvDev &ed,
                                              const float4 *__restrict__ env_rec,
                                              const float *__restrict__ q, int64_t n, int64_t ldq,
                                              const float *__restrict__ gcost,
                                              float *__restrict__ grad, int64_t ldg,
                                              float *__restrict__ cost_out, int cf,
                                              float *__restrict__ gslots) {
    extern __shared__ float4 lds_dyn[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int slot_floats = rb.n_links * 6 * kWave;
    float *slot_base, *lf;
    if (GSLOT) {
        slot_base = gslots + ((int64_t)blockIdx.x * (blockDim.x / kWave) + wave) * slot_floats;
        lf = reinterpret_cast<float *>(lds_dyn);
    } else {
        slot_base = reinterpret_cast<float *>(lds_dyn) + wave * slot_floats;
        lf = reinterpret_cast<float *>(lds_dyn) + slot_floats * (blockDim.x / kWave);
    }
    const StepCache sc = step_cache(lf, rb.n_slots, rb.dof, cf);
    float4 *lds_env = after_caches(lf, rb.n_slots, rb.dof, cf);
    if (STAGE) stage_env(lds_env, env_rec, ed.n_stage);
    const EnvView ev = make_view<STAGE>(ed, lds_env);
    LinkSlots slots{slot_base, lane};
    for (int l = 0; l < rb.n_links; ++l)
        for (int c = 0; c < 6; ++c) slots.at(l, c) = 0.0f;

    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    QState qs{q, ldq, active ? i : 0};
    bool finite = true;
    for (int j = 0; j < rb.dof; ++j) finite &= isfinite(qs(j));
    // the gradient's walk computes the cost too (in the forward walk's order): with cost_out it
    // is stored, and without gcost the gradient is d cost / d q itself
    const float cost = cost_walk<true>(rb, ev, ed, qs, sc, active && finite, slots);
    if (cost_out && active) cost_out[i] = finite ? cost : __builtin_nanf("");

    // suffix sums: child link totals into the parent (parents have smaller indices)
    for (int l = rb.n_links - 1; l >= 1; --l) {
        const int p = ld(rb.joints, l - 1).parent;
#pragma unroll
        for (int c = 0; c < 6; ++c) slots.at(p, c) += slots.at(l, c);
    }
    const float gc = active ? (gcost ? gcost[i] : 1.0f) : 0.0f;
    // one more forward pass for the joint frames P_j = T_parent(j) * M_j
    Frame T;
    frame_identity(T);
    int cur = 0;                               // link whose pose T holds
    for (int j = 0; j < rb.dof; ++j) {
        const JointRec J = ld(rb.joints, j);
        if (J.parent != cur) {
            // rebuild the parent's pose from the base along the restart path of the step
            // that poses link j+1 (stored with that step)
            frame_identity(T);
            for (int s = 0; s < rb.n_steps; ++s) {
                const StepRec S = ld(rb.steps, s);
                if (S.joint == j) {
                    for (int k = 0; k < S.restart_len; ++k) {
                        const int jj = ld(rb.paths, S.restart_off + k);
                        frame_joint(T, ld(rb.joints, jj), qs(jj));
                    }
                    break;
                }
            }
        }
        if (J.has_mount) frame_mount(T, J.m);
        const float zx = T.r[2], zy = T.r[5], zz = T.r[8];
        const float ox = T.p[0], oy = T.p[1], oz = T.p[2];
        const int l = j + 1;
        const float Fx = slots.at(l, 0), Fy = slots.at(l, 1), Fz = slots.at(l, 2);
        const float Mx = slots.at(l, 3) - (oy * Fz - oz * Fy);
        const float My = slots.at(l, 4) - (oz * Fx - ox * Fz);
        const float Mz = slots.at(l, 5) - (ox * Fy - oy * Fx);
        // revolute: z . (M - o x F); prismatic: the force along the slide axis, z . F
        const float g = J.prismatic ? fmaf(zx, Fx, fmaf(zy, Fy, zz * Fz))
                                    : fmaf(zx, Mx, fmaf(zy, My, zz * Mz));
        if (active) grad[j * ldg + i] = finite ? gc * g : __builtin_nanf("");
        frame_dh(T, J, qs(j));
        cur = l;
    }
}

template <int STAGE>
__global__ void __launch_bounds__(256)
    k_cost_bwd(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
               const float *__restrict__ q, int64_t n, int64_t ldq,
               const float *__restrict__ gcost, float *__restrict__ grad, int64_t ldg,
               float *__restrict__ cost_out, int cf) {
    cost_bwd_body<STAGE, false>(rb, ed, env_rec, q, n, ldq, gcost, grad, ldg, cost_out, cf,
                                nullptr);
}

// four waves per SIMD (at most 128 VGPRs): with the slots out of the LDS the registers are the
// occupancy limit
template <int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_cost_bwd_g(RobotDev rb, EnvDev ed, const float4 *__restrict__ env_rec,
                 const float *__restrict__ q, int64_t n, int64_t ldq,
                 const float *__restrict__ gcost, float *__restrict__ grad, int64_t ldg,
                 float *__restrict__ cost_out, int cf, float *__restrict__ gslots) {
    cost_bwd_body<STAGE, true>(rb, ed, env_rec, q, n, ldq, gcost, grad, ldg, cost_out, cf, gslots);
}

// ---------------------------------------------------------------------------------------------
// k nearest neighbours of samples in configuration space (the roadmap of a PRM, Sec. III-E:
// neighbours by the Euclidean norm).  One lane per query sample keeps a sorted top-K list in
// registers; candidate samples stream through LDS in tiles shared by the workgroup.  The
// squared distance is accumulated in joint order with separately rounded products and sums
// (no fused multiply-add), so the neighbour order is a well-defined FP32 result; equal
// distances go to the lower index.  Candidates with a non-finite distance are skipped; list
// slots left without a neighbour hold index -1 and distance +inf.
// ---------------------------------------------------------------------------------------------
#ifndef VK_KNN_TILE
#define VK_KNN_TILE 128
#endif
constexpr int kKnnTile = VK_KNN_TILE;

__device__ __forceinline__ bool knn_less(float d, int i, float e, int j) {
    return d < e || (d == e && i < j);
}

// Insert (s, c) into the sorted list (bd, bi) of length K if it beats the last entry.
template <int K>
__device__ __forceinline__ void knn_insert(float (&bd)[K], int (&bi)[K], float s, int c) {
    if (!knn_less(s, c, bd[K - 1], bi[K - 1])) return;
    bool done = false;
#pragma unroll
    for (int m = K - 1; m > 0; --m) {
        if (!done) {
            if (knn_less(s, c, bd[m - 1], bi[m - 1])) {
                bd[m] = bd[m - 1];
                bi[m] = bi[m - 1];
            } else {
                bd[m] = s;
                bi[m] = c;
                done = true;
            }
        }
    }
    if (!done) {
        bd[0] = s;
        bi[0] = c;
    }
}

// Partial lists: workgroup (tile, p) holds 64 queries (one wave) and scans the candidates of
// part p, [p n / parts, (p+1) n / parts), through LDS; each lane keeps the best K of that part
// in registers and writes them to part lists [parts][n][K] (index 0x7fffffff = none).  Splitting
// the candidates over parts gives the launch parts x n / 64 waves instead of n / 64.
// A candidate that beats its lane's current K-th goes to the lane's buffer in LDS first; the
// lanes merge their buffers into their lists when one lane's buffer is full (and at the end).
// Inserting one candidate at a time, a wave would run the sorted insertion for every
// candidate some lane accepts; with the buffers it runs as many insertions as its busiest lane
// accepted.  Every buffered candidate is still inserted in (distance, index) order, so the
// lists are the same.
#ifndef VK_KNN_BUF
#define VK_KNN_BUF 16
#endif
constexpr int kKnnBuf = VK_KNN_BUF;            // buffered candidates per lane

// DP: the dimension padded to a multiple of 4.  The query and the tile hold zeros past dim, and
// adding a zero term leaves a sum unchanged, so the padded sum equals the sum over dim terms
// in the same order; each candidate is read as DP / 4 16-byte LDS loads, with no branch per
// dimension.  DX (<= DP): the terms actually summed, the exact dimension where a launch knows
// it at compile time (7), else DP.
template <int K, int DP, int DX = DP>
__global__ void __launch_bounds__(64) k_knn_part(const float *__restrict__ x, int64_t n, int dim,
                                                 int parts, int32_t *__restrict__ pidx,
                                                 float *__restrict__ pd2) {
#pragma clang fp contract(off)                 // products and sums rounded separately
    extern __shared__ float4 lds4[];
    float4 *tile = lds4;                       // [kKnnTile][DP / 4]
    float *bufd = reinterpret_cast<float *>(lds4 + kKnnTile * (DP / 4));   // [kKnnBuf][64]
    int *bufi = reinterpret_cast<int *>(bufd + kKnnBuf * kWave);
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const int p = blockIdx.y;
    const int64_t c0 = n * p / parts, c1 = n * (p + 1) / parts;
    float xi[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) xi[j] = (active && j < dim) ? x[i * dim + j] : 0.0f;
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        bd[m] = INFINITY;
        bi[m] = 0x7fffffff;
    }
    int nb = 0;                                // this lane's buffered candidates
    const auto flush = [&]() {
        for (int b = 0; b < nb; ++b) knn_insert<K>(bd, bi, bufd[b * kWave + lane], bufi[b * kWave + lane]);
        nb = 0;
    };
    float *tile_f = reinterpret_cast<float *>(tile);
    for (int64_t t0 = c0; t0 < c1; t0 += kKnnTile) {
        const int tn = (int)(c1 - t0 < kKnnTile ? c1 - t0 : kKnnTile);
        __syncthreads();
        for (int v = threadIdx.x; v < tn * DP; v += blockDim.x) {
            const int t = v / DP, j = v - t * DP;
            tile_f[v] = j < dim ? x[(t0 + t) * dim + j] : 0.0f;
        }
        __syncthreads();
        for (int t = 0; t < tn; ++t) {
            float4 y[DP / 4];
#pragma unroll
            for (int q = 0; q < DP / 4; ++q) y[q] = tile[t * (DP / 4) + q];
            const float *yf = reinterpret_cast<const float *>(y);
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < DX; ++j) {       // plain operators: the pragma above keeps them apart
                const float d = xi[j] - yf[j];
                s = s + d * d;
            }
            // the part is scanned in increasing index order and its list holds only earlier
            // candidates, so a tie with the K-th entry never wins and `s < K-th distance` is
            // the whole acceptance test (false too for a NaN or infinite distance); buffered
            // candidates are inserted later with the full (distance, index) order
            const int c = (int)(t0 + t);
            if (active && c != i && s < bd[K - 1]) {
                bufd[nb * kWave + lane] = s;
                bufi[nb * kWave + lane] = c;
                ++nb;
            }
            if (wave_ballot(nb == kKnnBuf)) flush();
        }
    }
    flush();
    if (!active) return;
    const int64_t o = ((int64_t)p * n + i) * K;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        pidx[o + m] = bi[m];
        pd2[o + m] = bd[m];
    }
}

// Merge the parts' lists of each query into its k nearest (same order: distance, then index).
// A part's list is sorted, so once one of its entries does not beat the current K-th, none of
// the rest does either.
template <int K>
__global__ void __launch_bounds__(64) k_knn_merge(const int32_t *__restrict__ pidx,
                                                   const float *__restrict__ pd2, int64_t n,
                                                   int parts, int k, int32_t *__restrict__ idx,
                                                   float *__restrict__ d2out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        bd[m] = INFINITY;
        bi[m] = 0x7fffffff;
    }
    // each part's list is read whole (K / 4 16-byte loads of indices and of distances; K is a
    // multiple of 4 and every list starts on a 16-byte boundary), the next part's while this
    // one merges, instead of one dependent load per entry
    static_assert(K % 4 == 0, "list lengths are multiples of 4");
    int4 ci[K / 4], cn[K / 4];
    float4 di[K / 4], dn[K / 4];
    const auto load = [&](int p, int4 (&c)[K / 4], float4 (&d)[K / 4]) {
        const int64_t o = ((int64_t)p * n + i) * K;
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            c[q] = reinterpret_cast<const int4 *>(pidx + o)[q];
            d[q] = reinterpret_cast<const float4 *>(pd2 + o)[q];
        }
    };
    load(0, ci, di);
    for (int p = 0; p < parts; ++p) {
        if (p + 1 < parts) load(p + 1, cn, dn);
        const int *cc = reinterpret_cast<const int *>(ci);
        const float *dd = reinterpret_cast<const float *>(di);
        bool go = true;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            go = go && cc[m] != 0x7fffffff && knn_less(dd[m], cc[m], bd[K - 1], bi[K - 1]);
            if (go) knn_insert<K>(bd, bi, dd[m], cc[m]);
        }
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            ci[q] = cn[q];
            di[q] = dn[q];
        }
    }
#pragma unroll
    for (int m = 0; m < K; ++m)
        if (m < k) {
            const bool ok = bi[m] != 0x7fffffff;
            idx[i * k + m] = ok ? bi[m] : -1;
            d2out[i * k + m] = ok ? bd[m] : INFINITY;
        }
}

// ---------------------------------------------------------------------------------------------
// Tree primitives of a many-query RRT-Connect (Sec. III-E's planner, run for many queries in
// lockstep): every query q owns a tree of up to `cap` nodes, nodes[q][cap][dof], of which the
// first sizes[q] are in use.  The planner loop itself runs on the host; the edge checks are
// validate_edges.
// ---------------------------------------------------------------------------------------------

// Index of the node of tree[0 .. size) nearest to tg, by one wave (squared distance accumulated
// in joint order with separately rounded products and sums, ties to the lower index); -1 when
// size is 0.  Every lane returns the result.
__device__ int wave_nearest(const float *__restrict__ tree, int size, int dof,
                            const float *__restrict__ tg, int lane) {
#pragma clang fp contract(off)                 // products and sums rounded separately
    float best = INFINITY;
    int bi = 0x7fffffff;
    for (int v = lane; v < size; v += kWave) {
        float s = 0.0f;
        for (int j = 0; j < dof; ++j) {
            const float d = tree[(int64_t)v * dof + j] - tg[j];
            const float dd = d * d;
            s = s + dd;
        }
        if (knn_less(s, v, best, bi)) {
            best = s;
            bi = v;
        }
    }
    for (int m = 1; m < kWave; m <<= 1) {      // wave minimum of (distance, index)
        const float ob = __shfl_xor(best, m);
        const int oi = __shfl_xor(bi, m);
        if (knn_less(ob, oi, best, bi)) {
            best = ob;
            bi = oi;
        }
    }
    return bi == 0x7fffffff ? -1 : bi;
}

// Nearest tree node to targets[q] (one wave per query); -1 for an empty tree or an inactive
// query.
__global__ void __launch_bounds__(256) k_tree_nearest(const float *__restrict__ nodes,
                                                      const int32_t *__restrict__ sizes, int cap,
                                                      int dof, int64_t nq,
                                                      const float *__restrict__ targets,
                                                      const uint8_t *__restrict__ active,
                                                      int32_t *__restrict__ near) {
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (qi >= nq) return;                      // whole wave past the queries
    const bool on = !active || active[qi];
    const int size = on ? min(sizes[qi], cap) : 0;
    const int bi = wave_nearest(nodes + qi * (int64_t)cap * dof, size, dof, targets + qi * dof, lane);
    if (lane == 0) near[qi] = bi;
}

// Step from node a toward target tg by at most `step` (Euclidean): the factor f with
// q_new = a + f (tg - a), and whether tg lies within the step (then q_new = tg).  The squared
// length is accumulated in joint order with fused multiply-adds.
__device__ inline float steer_factor(const float *__restrict__ a, const float *__restrict__ tg,
                                     int dof, float step, bool &close) {
    float s = 0.0f;
    for (int j = 0; j < dof; ++j) {
        const float d = tg[j] - a[j];
        s = fmaf(d, d, s);
    }
    const float len = sqrtf(s);
    close = len <= step;
    return close ? 1.0f : step / len;
}

__device__ inline float steer_joint(float a, float tg, float f, bool close) {
    return close ? tg : fmaf(f, tg - a, a);
}

// Steer from node near[q] toward targets[q] by at most `step`: q_new = target when it is that
// close (reached[q] = 1), else near + d * (step / |d|).  Queries with near < 0 get reached = 0
// and q_new = target.
__global__ void k_tree_steer(const float *__restrict__ nodes, int cap, int dof, int64_t nq,
                             const int32_t *__restrict__ near, const float *__restrict__ targets,
                             float step, float *__restrict__ qnew, uint8_t *__restrict__ reached) {
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const float *tg = targets + qi * dof;
    float *o = qnew + qi * dof;
    const int ni = near[qi];
    if (ni < 0 || ni >= cap) {
        for (int j = 0; j < dof; ++j) o[j] = tg[j];
        reached[qi] = 0;
        return;
    }
    const float *a = nodes + (qi * (int64_t)cap + ni) * dof;
    bool close;
    const float f = steer_factor(a, tg, dof, step, close);
    for (int j = 0; j < dof; ++j) o[j] = steer_joint(a[j], tg[j], f, close);
    reached[qi] = close ? 1 : 0;
}

// Append qnew[q] to tree q with parent near[q] where ok[q] (and the tree has room); the new
// node's index goes to added[q] (-1 when nothing was added).
__global__ void k_tree_append(float *__restrict__ nodes, int32_t *__restrict__ parents,
                              int32_t *__restrict__ sizes, int cap, int dof, int64_t nq,
                              const float *__restrict__ qnew, const int32_t *__restrict__ near,
                              const uint8_t *__restrict__ ok, int32_t *__restrict__ added) {
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const int size = sizes[qi];
    const int ni = near[qi];
    if (!ok[qi] || ni < 0 || ni >= size || size >= cap) {
        added[qi] = -1;
        return;
    }
    float *dst = nodes + (qi * (int64_t)cap + size) * dof;
    for (int j = 0; j < dof; ++j) dst[j] = qnew[qi * dof + j];
    parents[qi * (int64_t)cap + size] = ni;
    sizes[qi] = size + 1;
    added[qi] = size;
}

// One extension of every query's tree toward its target, fused into one launch: the nearest
// node (as k_tree_nearest), the step toward the target (as k_tree_steer) and the edge to check,
// qnear[q] -> qnew[q].  A query that is inactive, or whose tree is empty, gets near = -1,
// reached = 0 and a zero-length edge at its tree's root (at the target for an empty tree).
// One wave per query; lanes write the joints.
__global__ void __launch_bounds__(256) k_rrt_extend(const float *__restrict__ nodes,
                                                    const int32_t *__restrict__ sizes, int cap,
                                                    int dof, int64_t nq,
                                                    const float *__restrict__ targets,
                                                    const uint8_t *__restrict__ active, float step,
                                                    float *__restrict__ qnear,
                                                    float *__restrict__ qnew,
                                                    int32_t *__restrict__ near,
                                                    uint8_t *__restrict__ reached) {
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (qi >= nq) return;                      // whole wave past the queries
    const float *tree = nodes + qi * (int64_t)cap * dof;
    const float *tg = targets + qi * dof;
    const int size = min(sizes[qi], cap);
    const int bi = active[qi] ? wave_nearest(tree, size, dof, tg, lane) : -1;
    float *on = qnear + qi * dof, *ow = qnew + qi * dof;
    if (bi < 0) {
        const float *p = size > 0 ? tree : tg;
        for (int j = lane; j < dof; j += kWave) on[j] = ow[j] = p[j];
        if (lane == 0) {
            near[qi] = -1;
            reached[qi] = 0;
        }
        return;
    }
    const float *a = tree + (int64_t)bi * dof;
    bool close;
    const float f = steer_factor(a, tg, dof, step, close);   // the same value in every lane
    for (int j = lane; j < dof; j += kWave) {
        on[j] = a[j];
        ow[j] = steer_joint(a[j], tg[j], f, close);
    }
    if (lane == 0) {
        near[qi] = bi;
        reached[qi] = close ? 1 : 0;
    }
}

// Bookkeeping after the edges of an extension of tree t were checked (flags[q] != 0: the edge
// collides), fused into one launch.  For each query with going[q] != 0: count its edge, and append
// qnew[q] (parent near[q]) when its edge is free, near[q] is a node and the tree has room;
// added[q] = the new node's index, else -1.  Then going[q] becomes:
//  - without from_added (the extension toward a sample): whether a node was added;
//  - with from_added (an extension toward the other tree's new node from_added[q]): whether a
//    node was added short of the target.  A node added at the target joins the trees: solved[q]
//    = 1, meet_this[q] = added[q], meet_from[q] = from_added[q].
// One thread per query.
__global__ void k_rrt_commit(float *__restrict__ nodes, int32_t *__restrict__ parents,
                             int32_t *__restrict__ sizes, int cap, int dof, int64_t nq,
                             const float *__restrict__ qnew, const int32_t *__restrict__ near,
                             const uint8_t *__restrict__ reached,
                             const uint8_t *__restrict__ flags, uint8_t *__restrict__ going,
                             int32_t *__restrict__ added, const int32_t *__restrict__ from_added,
                             int64_t *__restrict__ meet_this, int64_t *__restrict__ meet_from,
                             uint8_t *__restrict__ solved, unsigned long long *__restrict__ edges) {
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const bool act = going[qi] != 0;
    int ai = -1;
    if (act) {
        atomicAdd(edges, 1ull);
        const int size = sizes[qi];
        const int ni = near[qi];
        if (!flags[qi] && ni >= 0 && ni < size && size < cap) {
            float *dst = nodes + (qi * (int64_t)cap + size) * dof;
            for (int j = 0; j < dof; ++j) dst[j] = qnew[qi * dof + j];
            parents[qi * (int64_t)cap + size] = ni;
            sizes[qi] = size + 1;
            ai = size;
        }
    }
    added[qi] = ai;
    if (!from_added) {
        going[qi] = ai >= 0 ? 1 : 0;
        return;
    }
    const bool at = ai >= 0 && reached[qi];
    if (at) {
        meet_this[qi] = ai;
        meet_from[qi] = from_added[qi];
        solved[qi] = 1;
    }
    going[qi] = ai >= 0 && !reached[qi] ? 1 : 0;
}

// Undirected roadmap edges from kNN lists, one slot per (i, m): (i, j) for j = idx[i][m] when
// i < j or when i is not in j's list, else the hole (-1, -1); each edge appears exactly once.
__global__ void k_knn_pairs(const int32_t *__restrict__ idx, int64_t n, int k,
                            int32_t *__restrict__ pairs) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * k) return;
    const int64_t i = s / k;
    const int32_t j = idx[s];
    bool keep = j >= 0 && j < n && j != i;
    if (keep && j < i)
        for (int m = 0; m < k; ++m)
            if (idx[(int64_t)j * k + m] == i) keep = false;
    pairs[2 * s] = keep ? (int32_t)i : -1;
    pairs[2 * s + 1] = keep ? j : -1;
}

// ---------------------------------------------------------------------------------------------
// Randomized shortcutting of many paths at once (the path simplification of Sec. III-E): each
// round proposes K waypoint pairs per path, validates them all in one edge launch, and splices
// in one valid shortcut per path.  Paths are [P][M][dof] (waypoint w of path p is node p*M + w),
// lens [P] the waypoints in use.
// ---------------------------------------------------------------------------------------------
// Candidate k of path p from two random words: i uniform-ish in [0, len - 3], j in
// [i + 2, len - 1], as node indices; a path of fewer than 3 waypoints gets holes (-1, -1).
__global__ void k_shortcut_propose(const int32_t *__restrict__ lens, int64_t P, int M, int K,
                                   const uint32_t *__restrict__ rnd, int32_t *__restrict__ pairs) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P * K) return;
    const int64_t p = s / K;
    const int len = min(max(lens[p], 0), M);
    int32_t a = -1, b = -1;
    if (len >= 3) {
        const int i = (int)(rnd[2 * s] % (uint32_t)(len - 2));
        const int j = i + 2 + (int)(rnd[2 * s + 1] % (uint32_t)(len - i - 2));
        a = (int32_t)(p * M + i);
        b = (int32_t)(p * M + j);
    }
    pairs[2 * s] = a;
    pairs[2 * s + 1] = b;
}

// Per path: the valid candidate (flag 0) that skips the most waypoints (ties to the lower k) is
// spliced in: waypoints i+1 .. j-1 are removed and the tail moves down.  accepted[p] (optional)
// is 1 where a shortcut was taken.
__global__ void k_shortcut_apply(float *__restrict__ paths, int32_t *__restrict__ lens, int64_t P,
                                 int M, int dof, int K, const int32_t *__restrict__ pairs,
                                 const uint8_t *__restrict__ flags, uint8_t *__restrict__ accepted) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int len = min(max(lens[p], 0), M);
    int bi = -1, bj = -1;
    for (int k = 0; k < K; ++k) {
        const int64_t c = p * K + k;
        const int32_t a = pairs[2 * c], b = pairs[2 * c + 1];
        if (a < 0 || b < 0 || flags[c] != 0) continue;
        const int i = (int)(a - p * M), j = (int)(b - p * M);
        if (i < 0 || j >= len || j - i < 2) continue;
        if (j - i > bj - bi) {
            bi = i;
            bj = j;
        }
    }
    if (bi >= 0) {
        float *w = paths + p * (int64_t)M * dof;
        for (int m = bj; m < len; ++m)
            for (int d = 0; d < dof; ++d) w[(int64_t)(bi + 1 + m - bj) * dof + d] = w[(int64_t)m * dof + d];
        lens[p] = len - (bj - bi - 1);
    }
    if (accepted) accepted[p] = bi >= 0 ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// Host-side launchers (called from the C-ABI layer).
// ---------------------------------------------------------------------------------------------
hipError_t launch_fk_spheres(const RobotDev &rb, const float *q, int64_t n, int64_t ldq,
                             float *out, int64_t ldc, hipStream_t s) {
    const int bs = 256;
    const int64_t grid = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_fk_spheres, dim3((unsigned)grid), dim3(bs), 0, s, rb, q, n, ldq, out, ldc);
    return hipGetLastError();
}

size_t walk_lds_bytes(const RobotDev &rb, int block, int cf) {
    return (size_t)(block / kWave) * step_cache_floats(rb.n_slots, rb.dof, cf) * sizeof(float);
}

static size_t device_max_lds();

int walk_block(const RobotDev &rb, int want) {
    const size_t max_lds = device_max_lds();
    int bs = want;
    while (bs > kWave && walk_lds_bytes(rb, bs, 0) > max_lds) bs -= kWave;
    return bs;
}

// Resident workgroups per CU of a kernel at a block size and dynamic LDS (memoised: the
// runtime query is not free and launches repeat with the same shapes).
static int resident_blocks(const void *kernel, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t>, int> memo;
    const auto key = std::make_tuple(kernel, block, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess) n = 0;
    std::lock_guard<std::mutex> lk(mu);
    memo[key] = n;
    return n;
}

// Staging mode of a launch (see make_view).  ed.n_stage arrives as the largest prefix that fits
// the LDS; a prefix is staged only if it costs no resident workgroups against reading every
// record from global memory: when the per-wave walk caches already fill the LDS, staging the
// records would trade occupancy for latency, and occupancy matters more here.  On return
// ed.n_stage is the prefix the chosen mode stages.
static int pick_stage(EnvDev &ed, const void *k0, const void *k1, const void *k2, int block,
                      size_t base) {
    const int occ0 = resident_blocks(k0, block, base);
    if (ed.n_stage > ed.off_cell && resident_blocks(k2, block, base + (size_t)ed.n_stage * 16) >= occ0)
        return 2;
    if (ed.off_cell > 0 && ed.n_stage >= ed.off_cell &&
        resident_blocks(k1, block, base + (size_t)ed.off_cell * 16) >= occ0) {
        ed.n_stage = ed.off_cell;
        return 1;
    }
    ed.n_stage = 0;
    return 0;
}

// LDS a workgroup may use on the current device (memoised per device).
static size_t device_max_lds() {
    static std::mutex mu;
    static std::map<int, size_t> memo;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(dev);
    if (it != memo.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 64 * 1024;
    return memo[dev] = (size_t)v;
}

// Optional parts of the walk cache (see StepCache), in the order of preference: the capsule
// halves (a second self-block gate before posing) ahead of the joint values (cheaper
// re-posing).  A launch takes the option, with its best staging mode, that keeps the most
// resident workgroups, then one that stages records, then the earlier option.
#ifndef VK_CACHE_PARTS
#define VK_CACHE_PARTS (kCacheCaps | kCacheJoints)   // the parts a launch may use
#endif
static const int kCacheOrder[4] = {kCacheCaps | kCacheJoints, kCacheCaps, kCacheJoints, 0};

// Launch KERNEL<stage, ...> with the cache parts and the staging mode chosen as above; the
// launcher defines grid_, block_, lds_(cf) (dynamic LDS before staging with cache parts cf),
// max_lds_ and ARGS_ (which passes cf).
#define VK_STAGED(KERNEL, ...)                                                                  \
    {                                                                                           \
        const void *k_[3] = {reinterpret_cast<const void *>(&KERNEL<0 __VA_ARGS__>),           \
                             reinterpret_cast<const void *>(&KERNEL<1 __VA_ARGS__>),           \
                             reinterpret_cast<const void *>(&KERNEL<2 __VA_ARGS__>)};          \
        EnvDev ed = ed_in;                                                                      \
        int cf = 0, mode = 0, best_ = -1;                                                       \
        for (int o_ = 0; o_ < 4; ++o_) {                                                        \
            const int c_ = kCacheOrder[o_];                                                     \
            if ((c_ & ~(VK_CACHE_PARTS)) != 0 || lds_(c_) > max_lds_) continue;                 \
            EnvDev e_ = ed_in;                                                                  \
            const int m_ = pick_stage(e_, k_[0], k_[1], k_[2], (int)block_.x, lds_(c_));       \
            const int r_ = resident_blocks(k_[m_], (int)block_.x, lds_(c_) + (size_t)e_.n_stage * 16); \
            if (r_ > best_ || (r_ == best_ && m_ > 0 && mode == 0)) {                           \
                best_ = r_;                                                                     \
                cf = c_;                                                                        \
                mode = m_;                                                                      \
                ed = e_;                                                                        \
            }                                                                                   \
        }                                                                                       \
        if (best_ < 0) ed.n_stage = 0;                                                          \
        const size_t sh_ = lds_(cf) + (size_t)ed.n_stage * 16;                                  \
        switch (mode) {                                                                         \
        case 0: hipLaunchKernelGGL((KERNEL<0 __VA_ARGS__>), grid_, block_, sh_, s, ARGS_); break; \
        case 1: hipLaunchKernelGGL((KERNEL<1 __VA_ARGS__>), grid_, block_, sh_, s, ARGS_); break; \
        default: hipLaunchKernelGGL((KERNEL<2 __VA_ARGS__>), grid_, block_, sh_, s, ARGS_); break; \
        }                                                                                       \
    }

// Link steps pass 1 of the two-pass state validation tests, for a fraction num/den of the
// robot's steps (0: one pass).  The kernels take the number of the first test of that step.
int states_split(const RobotDev &rb, int64_t n, int num, int den) {
    if (num <= 0 || den <= 0) return 0;
    const int split = (int)((int64_t)rb.n_steps * num / den);
    if (split <= 0 || split >= rb.n_steps || n >= (int64_t(1) << 31)) return 0;
    return split;
}

size_t states_scratch_bytes(int64_t n) { return 256 + (size_t)n * sizeof(int32_t); }

// Scratch of the allocation-free state validation: the survivor counter and list of up to
// kNoAllocStates states, in a file-scope device array that each GPU the library runs on holds
// until the process ends.  Host code never uses the array's name as an address (on the host it
// names a stand-in, not device memory): noalloc_scratch() looks up each device's own address
// once, with that device current, and hands that out.
constexpr int64_t kNoAllocStates = int64_t(1) << 22;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocStates * sizeof(int32_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int64_t noalloc_max_states() { return kNoAllocStates; }

hipError_t noalloc_scratch(void **ptr) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess) return err;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

hipError_t launch_validate_states(const RobotDev &rb, const EnvDev &ed_in, const float *q, int64_t n,
                                  int64_t ldq, uint8_t *out, int split, void *scratch,
                                  hipStream_t s, const StepRanges *ranges) {
    const int bs = walk_block(rb, 256);
    const auto lds_ = [&](int c) { return walk_lds_bytes(rb, bs, c); };
    const size_t max_lds_ = device_max_lds();
    if (!scratch) split = 0;
    if (split == 0) {
        StepRanges r;
        r.n = 1;
        r.b[0] = 0;
        r.b[1] = rb.n_steps;
        if (ranges && ranges->n > 1) {
            r = *ranges;
            hipLaunchKernelGGL(k_zero_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n);
        }
        const dim3 grid_((unsigned)((n + bs - 1) / bs), (unsigned)r.n), block_(bs);
#define ARGS_ rb, ed, ed.rec, q, n, ldq, out, cf, r
        VK_STAGED(k_validate_states)
#undef ARGS_
        return hipGetLastError();
    }
    const dim3 grid_((unsigned)((n + bs - 1) / bs)), block_(bs);
    unsigned long long *n_surv = static_cast<unsigned long long *>(scratch);
    int32_t *surv = reinterpret_cast<int32_t *>(static_cast<char *>(scratch) + 256);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, n_surv, 0ull, 1, 1);
#define ARGS_ rb, ed, ed.rec, q, n, ldq, out, cf, split, surv, n_surv
    VK_STAGED(k_validate_states_screen)
#undef ARGS_
#define ARGS_ rb, ed, ed.rec, q, ldq, out, cf, split, surv, n_surv
    VK_STAGED(k_validate_states_rest)
#undef ARGS_
    return hipGetLastError();
}

int knn_parts(int64_t n) {
    const int64_t tiles = (n + kWave - 1) / kWave;
    int64_t p = (2048 + tiles - 1) / tiles;    // aim at ~2,048 waves
    p = std::min<int64_t>(p, std::max<int64_t>(1, n / kWave));
    return (int)std::max<int64_t>(1, std::min<int64_t>(p, 64));
}

static int knn_list_len(int k) { return k <= 4 ? 4 : k <= 8 ? 8 : k <= 12 ? 12 : k <= 16 ? 16 : 32; }

size_t knn_workspace_bytes(int64_t n, int k) {
    return (size_t)knn_parts(n) * n * knn_list_len(k) * (sizeof(int32_t) + sizeof(float));
}

// parts(n) <= ceil(2048 / ceil(n / 64)) <= 2048 * 64 / n + 1, so parts(n) * n <= 131072 + n; a
// count below 64 has one part
size_t knn_workspace_bound(int64_t max_n, int k) {
    if (max_n <= 0) return 0;
    const int64_t pn = std::max<int64_t>(64, 2048 * (int64_t)kWave + max_n);
    return (size_t)pn * knn_list_len(k) * (sizeof(int32_t) + sizeof(float));
}

hipError_t launch_knn(const float *x, int64_t n, int dim, int k, int32_t *idx, float *d2,
                      void *workspace, hipStream_t s) {
    const int parts = knn_parts(n), K = knn_list_len(k);
    int32_t *pidx = static_cast<int32_t *>(workspace);
    float *pd2 = reinterpret_cast<float *>(pidx + (size_t)parts * n * K);
    const dim3 grid_((unsigned)((n + kWave - 1) / kWave), (unsigned)parts), block_(kWave);
    const int dp = dim <= 4 ? 4 : dim <= 8 ? 8 : dim <= 16 ? 16 : dim <= 32 ? 32 : 64;
    const size_t sh = (size_t)dp * kKnnTile * sizeof(float) + (size_t)kKnnBuf * kWave * 8;
    const dim3 mgrid((unsigned)((n + kWave - 1) / kWave)), mblock(kWave);
#define VK_KNN(KK, D)                                                                              \
    do {                                                                                           \
        if (D == 8 && dim == 7)                                                                    \
            hipLaunchKernelGGL((k_knn_part<KK, D, (D == 8 ? 7 : D)>), grid_, block_, sh, s, x, n,    \
                               dim, parts, pidx, pd2);                                             \
        else                                                                                       \
            hipLaunchKernelGGL((k_knn_part<KK, D>), grid_, block_, sh, s, x, n, dim, parts, pidx,   \
                               pd2);                                                               \
        hipLaunchKernelGGL((k_knn_merge<KK>), mgrid, mblock, 0, s, pidx, pd2, n, parts, k, idx, d2); \
    } while (0)
#define VK_KNN_K(D)                                                                               \
    do {                                                                                           \
        if (K == 4) VK_KNN(4, D);                                                                  \
        else if (K == 8) VK_KNN(8, D);                                                             \
        else if (K == 12) VK_KNN(12, D);                                                           \
        else if (K == 16) VK_KNN(16, D);                                                           \
        else VK_KNN(32, D);                                                                        \
    } while (0)
    switch (dp) {
    case 4: VK_KNN_K(4); break;
    case 8: VK_KNN_K(8); break;
    case 16: VK_KNN_K(16); break;
    case 32: VK_KNN_K(32); break;
    default: VK_KNN_K(64); break;
    }
#undef VK_KNN_K
#undef VK_KNN
    return hipGetLastError();
}

hipError_t launch_tree_nearest(const float *nodes, const int32_t *sizes, int cap, int dof,
                               int64_t nq, const float *targets, const uint8_t *active,
                               int32_t *near, hipStream_t s) {
    const int wpb = 4;
    hipLaunchKernelGGL(k_tree_nearest, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(wpb * kWave), 0,
                       s, nodes, sizes, cap, dof, nq, targets, active, near);
    return hipGetLastError();
}

hipError_t launch_tree_steer(const float *nodes, int cap, int dof, int64_t nq, const int32_t *near,
                             const float *targets, float step, float *qnew, uint8_t *reached,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_tree_steer, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nodes,
                       cap, dof, nq, near, targets, step, qnew, reached);
    return hipGetLastError();
}

hipError_t launch_tree_append(float *nodes, int32_t *parents, int32_t *sizes, int cap, int dof,
                              int64_t nq, const float *qnew, const int32_t *near,
                              const uint8_t *ok, int32_t *added, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_append, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nodes,
                       parents, sizes, cap, dof, nq, qnew, near, ok, added);
    return hipGetLastError();
}

hipError_t launch_rrt_extend(const float *nodes, const int32_t *sizes, int cap, int dof,
                             int64_t nq, const float *targets, const uint8_t *active, float step,
                             float *qnear, float *qnew, int32_t *near, uint8_t *reached,
                             hipStream_t s) {
    const int wpb = 4;
    hipLaunchKernelGGL(k_rrt_extend, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(wpb * kWave), 0,
                       s, nodes, sizes, cap, dof, nq, targets, active, step, qnear, qnew, near,
                       reached);
    return hipGetLastError();
}

hipError_t launch_rrt_commit(float *nodes, int32_t *parents, int32_t *sizes, int cap, int dof,
                             int64_t nq, const float *qnew, const int32_t *near,
                             const uint8_t *reached, const uint8_t *flags, uint8_t *going,
                             int32_t *added, const int32_t *from_added, int64_t *meet_this,
                             int64_t *meet_from, uint8_t *solved, uint64_t *edges,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_rrt_commit, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nodes,
                       parents, sizes, cap, dof, nq, qnew, near, reached, flags, going, added,
                       from_added, meet_this, meet_from, solved, (unsigned long long *)edges);
    return hipGetLastError();
}

hipError_t launch_knn_pairs(const int32_t *idx, int64_t n, int k, int32_t *pairs, hipStream_t s) {
    const int bs = 256;
    hipLaunchKernelGGL(k_knn_pairs, dim3((unsigned)((n * k + bs - 1) / bs)), dim3(bs), 0, s, idx,
                       n, k, pairs);
    return hipGetLastError();
}

hipError_t launch_shortcut_propose(const int32_t *lens, int64_t P, int M, int K,
                                  const uint32_t *rnd, int32_t *pairs, hipStream_t s) {
    const int64_t n = P * K;
    hipLaunchKernelGGL(k_shortcut_propose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lens,
                       P, M, K, rnd, pairs);
    return hipGetLastError();
}

hipError_t launch_shortcut_apply(float *paths, int32_t *lens, int64_t P, int M, int dof, int K,
                                const int32_t *pairs, const uint8_t *flags, uint8_t *accepted,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_shortcut_apply, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, paths,
                       lens, P, M, dof, K, pairs, flags, accepted);
    return hipGetLastError();
}

hipError_t launch_reset_queue(unsigned long long *queue, hipStream_t s, uint8_t *flags,
                              int64_t n_flags) {
    if (flags && n_flags > 0)
        hipLaunchKernelGGL(k_reset_queue_flags, dim3((unsigned)((n_flags + 255) / 256)), dim3(256), 0,
                           s, queue, flags, n_flags);
    else
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, queue, 0ull, kQueues, kQueueWords);
    return hipGetLastError();
}

// Items per ticket of a persistent launch: about `tickets` tickets per wave (a launch setting,
// 8 by default) keeps the dynamic balance fine while bounding the number of queue atomics.
static int work_chunk(int64_t n_items, int grid, int block, int tickets) {
    const int64_t waves = (int64_t)grid * (block / kWave);
    const int64_t c = n_items / (waves * std::max(tickets, 1));
    return (int)(c < 1 ? 1 : (c > 64 ? 64 : c));
}

hipError_t launch_validate_edges(const RobotDev &rb, const EnvDev &ed_in, const EdgeSrc &src,
                                 int64_t n_edges, float res, uint8_t *out,
                                 unsigned long long *queue, int grid, int block, int tickets,
                                 int parts, int tparts, hipStream_t s, unsigned long long *flops) {
    const dim3 grid_(grid), block_(block);
    const auto lds_ = [&](int c) { return walk_lds_bytes(rb, block, c); };
    const size_t max_lds_ = device_max_lds();
    const bool multi = parts > 1 || tparts > 1;   // flags zeroed with the queue reset
    const int chunk = work_chunk(n_edges * parts * tparts, grid, block, tickets);
#define ARGS_ rb, ed, ed.rec, src, n_edges, res, out, queue, chunk, flops, cf, parts, tparts
    if (multi) {
        if (flops) {
            VK_STAGED(k_validate_edges, , true, true)
        } else {
            VK_STAGED(k_validate_edges, , false, true)
        }
    } else {
        if (flops) {
            VK_STAGED(k_validate_edges, , true, false)
        } else {
            VK_STAGED(k_validate_edges, , false, false)
        }
    }
#undef ARGS_
    return hipGetLastError();
}

// Resident workgroups per CU of a kernel compiled for one robot (memoised like resident_blocks).
static int resident_blocks_fn(hipFunction_t f, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<hipFunction_t, int, size_t>, int> memo;
    const auto key = std::make_tuple(f, block, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    int n = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds) != hipSuccess) n = 0;
    std::lock_guard<std::mutex> lk(mu);
    memo[key] = n;
    return n;
}

hipError_t launch_validate_edges_spec(const SpecEdgeKernels &K, const RobotDev &rb,
                                      const EnvDev &ed_in, const EdgeSrc &src, int64_t n_edges,
                                      float res, uint8_t *out, unsigned long long *queue, int grid,
                                      int block, int tickets, int parts, int tparts,
                                      hipStream_t s, unsigned long long *flops) {
    const hipFunction_t *fk = flops ? K.counted : K.edges;
    const size_t max_lds = device_max_lds();
    // the specialised kernels are compiled in the multi-part form, which stores only the 1s:
    // the flags were zeroed with the queue reset
    const int chunk = work_chunk(n_edges * parts * tparts, grid, block, tickets);
    // the cache parts and the staging mode as VK_STAGED chooses them for the library's kernels
    EnvDev ed = ed_in;
    int cf = 0, mode = 0, best = -1;
    for (int o = 0; o < 4; ++o) {
        const int c = kCacheOrder[o];
        const size_t base = walk_lds_bytes(rb, block, c);
        if ((c & ~(VK_CACHE_PARTS)) != 0 || base > max_lds) continue;
        EnvDev e = ed_in;
        const int occ0 = resident_blocks_fn(fk[0], block, base);
        int m = 0;
        if (e.n_stage > e.off_cell && resident_blocks_fn(fk[2], block, base + (size_t)e.n_stage * 16) >= occ0) {
            m = 2;
        } else if (e.off_cell > 0 && e.n_stage >= e.off_cell &&
                   resident_blocks_fn(fk[1], block, base + (size_t)e.off_cell * 16) >= occ0) {
            e.n_stage = e.off_cell;
            m = 1;
        } else {
            e.n_stage = 0;
        }
        const int r = resident_blocks_fn(fk[m], block, base + (size_t)e.n_stage * 16);
        if (r > best || (r == best && m > 0 && mode == 0)) {
            best = r;
            cf = c;
            mode = m;
            ed = e;
        }
    }
    if (best < 0) ed.n_stage = 0;
    const size_t sh = walk_lds_bytes(rb, block, cf) + (size_t)ed.n_stage * 16;
    RobotDev rb_ = rb;
    const float4 *rec = ed.rec;
    EdgeSrc src_ = src;
    void *args[] = {&rb_, &ed, &rec, &src_, &n_edges, &res, &out, &queue,
                    const_cast<int *>(&chunk), &flops, &cf, &parts, &tparts};
    return hipModuleLaunchKernel(fk[mode], (unsigned)grid, 1, 1, (unsigned)block, 1, 1, (unsigned)sh,
                                 s, args, nullptr);
}

hipError_t launch_validate_edge_one(const RobotDev &rb, const EnvDev &ed_in, const EdgeSrc &src,
                                    int64_t e, float res, uint8_t *out, hipStream_t s) {
    const dim3 grid_(1), block_(kWave);
    const auto lds_ = [&](int c) { return walk_lds_bytes(rb, kWave, c); };
    const size_t max_lds_ = device_max_lds();
#define ARGS_ rb, ed, ed.rec, src, e, res, out, cf
    VK_STAGED(k_validate_edge_one)
#undef ARGS_
    return hipGetLastError();
}

hipError_t launch_cost_fwd(const RobotDev &rb, const EnvDev &ed_in, const float *q, int64_t n,
                           int64_t ldq, float *cost, hipStream_t s) {
    const int bs = walk_block(rb, 256);
    const dim3 grid_((unsigned)((n + bs - 1) / bs)), block_(bs);
    const auto lds_ = [&](int c) { return walk_lds_bytes(rb, bs, c); };
    const size_t max_lds_ = device_max_lds();
#define ARGS_ rb, ed, ed.rec, q, n, ldq, cost, cf
    VK_STAGED(k_cost_fwd)
#undef ARGS_
    return hipGetLastError();
}

size_t cost_bwd_slot_bytes(const RobotDev &rb, int block, int cf) {
    return (size_t)rb.n_links * 6 * kWave * sizeof(float) * (block / kWave) +
           walk_lds_bytes(rb, block, cf);
}

size_t cost_bwd_global_slot_bytes(const RobotDev &rb, int64_t n, int block) {
    const int64_t blocks = (n + block - 1) / block;
    return (size_t)blocks * (block / kWave) * rb.n_links * 6 * kWave * sizeof(float);
}

int cost_bwd_lds_waves_per_cu(const RobotDev &rb, int block) {
    return resident_blocks(reinterpret_cast<const void *>(&k_cost_bwd<1>), block,
                           cost_bwd_slot_bytes(rb, block, 0)) *
           (block / kWave);
}

hipError_t launch_cost_bwd(const RobotDev &rb, const EnvDev &ed_in, const float *q, int64_t n,
                           int64_t ldq, const float *gcost, float *grad, int64_t ldg, int block,
                           hipStream_t s, float *cost, float *gslots) {
    const dim3 grid_((unsigned)((n + block - 1) / block)), block_(block);
    const size_t max_lds_ = device_max_lds();
    if (gslots) {
        const auto lds_ = [&](int c) { return walk_lds_bytes(rb, block, c); };
#define ARGS_ rb, ed, ed.rec, q, n, ldq, gcost, grad, ldg, cost, cf, gslots
        VK_STAGED(k_cost_bwd_g)
#undef ARGS_
        return hipGetLastError();
    }
    const auto lds_ = [&](int c) { return cost_bwd_slot_bytes(rb, block, c); };
#define ARGS_ rb, ed, ed.rec, q, n, ldq, gcost, grad, ldg, cost, cf
    VK_STAGED(k_cost_bwd)
#undef ARGS_
    return hipGetLastError();
}
#undef VK_STAGED

void fill_node(KernelNode &L, unsigned long long *p, unsigned long long v, int n, int stride) {
    L.fn = reinterpret_cast<const void *>(&k_fill_u64);
    L.grid = dim3(1);
    L.block = dim3(64);
    L.shmem = 0;
    L.fill = {p, v, n, stride};
    L.args[0] = &L.fill.p;
    L.args[1] = &L.fill.v;
    L.args[2] = &L.fill.n;
    L.args[3] = &L.fill.stride;
}

void edge_batch_node(KernelNode &L, const BatchSet *sets, const int32_t *edge_set, int n_sets,
                     int64_t total, float res, unsigned long long *queue, int grid, int block,
                     int tickets, int max_slots, int max_dof) {
    // cache parts as for the other walks (no staging here: the records change per set)
    const void *k = reinterpret_cast<const void *>(&k_validate_edge_batch);
    const size_t waves = (size_t)(block / kWave), max_lds = device_max_lds();
    int cf = 0, best = -1;
    for (int o = 0; o < 4; ++o) {
        const int c = kCacheOrder[o];
        const size_t bytes = waves * step_cache_floats(max_slots, max_dof, c) * sizeof(float);
        if ((c & ~(VK_CACHE_PARTS)) != 0 || bytes > max_lds) continue;
        const int r = resident_blocks(k, block, bytes);
        if (r > best) {
            best = r;
            cf = c;
        }
    }
    const int floats = step_cache_floats(max_slots, max_dof, cf);
    L.fn = k;
    L.grid = dim3(grid);
    L.block = dim3(block);
    L.shmem = waves * floats * sizeof(float);
    auto &a = L.batch;
    a.sets = sets;
    a.edge_set = edge_set;
    a.n_sets = n_sets;
    a.total = total;
    a.res = res;
    a.qa = a.qb = nullptr;
    a.out = nullptr;
    a.queue = queue;
    a.chunk = work_chunk(total, grid, block, tickets);
    a.floats = floats;
    a.cf = cf;
    void **v = L.args;
    v[0] = &a.sets;
    v[1] = &a.edge_set;
    v[2] = &a.n_sets;
    v[3] = &a.total;
    v[4] = &a.res;
    v[5] = &a.qa;
    v[6] = &a.qb;
    v[7] = &a.out;
    v[8] = &a.queue;
    v[9] = &a.chunk;
    v[10] = &a.floats;
    v[11] = &a.cf;
}

}  // namespace vk
