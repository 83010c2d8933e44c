// Device-resident records shared by the host runtime (vk_api.cpp) and the kernels.
//
// The host turns a robot description into a small uniform "program" that every lane of a
// wavefront walks in lock-step: a list of link steps in topological order (pose a link,
// place its spheres, test them, then test the self pairs that this link completes).  This
// is the GPU counterpart of the straight-line, topologically reordered FK + collision code
// the paper generates per robot (Sec. III-B tracing compiler, Sec. III-D interleaving): the
// control flow depends only on the robot, so it is identical in every lane and all of its
// data is read with wave-uniform (scalar) loads.
#pragma once
#include <stdint.h>

namespace vk {

constexpr int kWave = 64;          // CDNA wavefront width: one lane per configuration
constexpr int kSpl = 8;            // spheres held in registers per link step
// Work queues of the persistent launches: kQueues 64-bit counters, kQueueWords words apart
// (4 KiB, so the counters sit in different memory channels).
constexpr int kQueues = 8;
constexpr int kQueueWords = 512;
constexpr size_t kQueueBytes = (size_t)kQueues * kQueueWords * 8;
constexpr int kMaxDof = 64;
// Most states one edge may be discretised into.  A longer edge (a computed count that
// saturates, or an explicit count above this) is not validated and is reported as colliding;
// below it a state index and its interpolation parameter stay exact in 32-bit arithmetic.
constexpr int kMaxEdgeStates = 1 << 24;

// Twist codes: the paper's tracing compiler folds constant sin/cos of the DH twist; the
// common twists 0 and +-90 degrees are folded the same way here (a uniform branch picks the
// specialised update).
enum Twist : int32_t { kTwist0 = 0, kTwistP90 = 1, kTwistM90 = 2, kTwistGeneral = 3 };

struct JointRec {                  // 96 bytes
    float a, d, ca, sa;            // DH length, offset, cos/sin of twist
    float theta_off;
    float s_off, c_off;            // sin/cos of theta_off (the fixed angle of a prismatic joint)
    int32_t twist;                 // Twist
    int32_t has_mount;             // 0: mount is identity
    int32_t parent;                // link the joint hangs off
    int32_t prismatic;             // 1: slides along z by q (offset d + q), 0: turns by q
    float m[12];                   // mount, row-major 3x4
    int32_t index;                 // the joint's own index (copies of the record carry it)
};

// One link step.  If `joint` >= 0 the step first poses link joint+1: when `restart_len` >= 0
// the parent's pose is rebuilt from the base by applying the `restart_len` joints listed at
// paths[restart_off...] (a tree branch), otherwise the step continues from the previous
// step's pose (serial chain).  A link with more than kSpl spheres is split into several steps;
// the later ones have joint = -1 and reuse the pose.
struct StepRec {                   // 192 bytes
    int32_t joint;
    int32_t restart_off, restart_len;
    int32_t sph_first, sph_count;  // fine spheres of this step (<= kSpl)
    int32_t blk_first, blk_count;  // self-collision blocks completed by this step
    int32_t link;
    float coarse[4];               // bounding sphere of the step's spheres, link frame
    // Bounding capsule of the step's spheres (link frame): the segment c - h .. c + h about the
    // bounding sphere's centre c, radius cap_r (padded by 1 mm: it only gates self blocks, and
    // the padding covers the FP32 rounding of the segment distance).  cap_rq adds the bound of
    // the error of h stored in half precision (how an earlier step's capsule is kept per lane).
    // cap_uu = |2h|^2 and cap_inv = 1 / cap_uu (0 if h = 0).
    float cap_h[3];
    float cap_r, cap_rq, cap_uu, cap_inv;
    int32_t slot;                  // walk-cache slot of this step's bounds, -1 if no later
                                   // step's self block reads them
    float pad[4];
    // a copy of joints[joint] (when joint >= 0): the walk reads it with the step's own record
    // instead of waiting for the step's joint index before loading it
    JointRec jr;
};
static_assert(sizeof(StepRec) == 192, "StepRec layout");

// Parts of the walk cache a launch includes besides the bounding-sphere centres.
constexpr int kCacheJoints = 1;     // two floats per joint and lane
constexpr int kCacheCaps = 2;       // the capsule half-vector, two floats per slot and lane

// Floats of LDS per wave for the walk cache: per slot and lane the link bounding sphere's
// centre (3) and, with kCacheCaps, the capsule half-vector as halves (2); with kCacheJoints
// also two per joint and lane.  A launch leaves parts out when their LDS would cost resident
// waves.
__host__ __device__ constexpr int step_cache_floats(int n_slots, int dof, int cf) {
    return (n_slots * ((cf & kCacheCaps) ? 5 : 3) + ((cf & kCacheJoints) ? dof * 2 : 0)) * kWave;
}

// Self pairs between this step's spheres and the spheres of one earlier step (on link A).  The
// earlier step's link bounding sphere and bounding capsule (their world centre and half-vector
// are kept per lane in LDS) gate the block; only then is A posed into a second register frame,
// continuing from the frame's current link when that link is an ancestor of A (anc bits), else
// from the base along the full path of joints.
struct BlockRec {                  // 48 bytes
    int32_t step_a;                // earlier step
    int32_t path_off, path_len;    // joints from the base to link A, base-most first
    int32_t ent_first, ent_count;
    int32_t link;                  // A
    uint32_t anc_lo, anc_hi;       // bit l-1: link l (>= 1) is a proper ancestor of A
    // copies from the earlier step's record, so that the gates need no second dependent load:
    // its walk-cache slot, its bounding-sphere radius and its capsule gate radius (cap_rq)
    int32_t slot_a;
    float ra, rqa;
    float pad;
};
static_assert(sizeof(BlockRec) == 48, "BlockRec layout");

// One earlier sphere t of a block and the mask of this step's spheres it is paired with.
struct EntryRec {                  // 64 bytes (one scalar load)
    float x, y, z, r;              // centre in A's frame, radius
    uint32_t mask;                 // bit k: paired with the step's k-th sphere
    float gate2;                   // (r + R)^2, R the step's link bounding radius (rounded up)
    float nhr2;                    // -r^2 / 2
    float pad;
    float rr[kSpl];                // r * r_k for paired spheres k, -inf otherwise
};

struct RobotDev {
    const JointRec *joints;
    const StepRec *steps;
    const BlockRec *blocks;
    const EntryRec *entries;
    const int32_t *paths;
    const JointRec *path_recs;     // path_recs[i] = joints[paths[i]]: one load per path joint
    const float4 *spheres;         // [S] centre (link frame), radius
    const int32_t *sphere_step;    // [S] step index of each sphere (cost backward)
    int32_t dof, n_steps, n_spheres, n_links;
    int32_t n_slots;               // steps with a walk-cache slot
    int32_t n_tests;               // the walk's tests: n_steps environment parts + the blocks
};

// Environment.  Primitive records, packed as float4 in one buffer:
//   off_sph   spheres   1 x float4: (centre, radius)
//   off_cap   capsules  2 x float4: (p0, radius), (u = p1 - p0, 1 / (u . u) or 0)
//   off_cyl   cylinders 2 x float4: (centre, half height), (unit axis, radius)
//   off_box   boxes     4 x float4: (col_0 of R, e_0), (col_1, e_1), (col_2, e_2), (centre, 0)
//   off_cell  point-grid cell index (cell_start, n_cells + 1 ints, four per record)
//   off_vdist voxel distance bytes (16 per record)
// A launch stages a prefix of the buffer in LDS: the primitives and the cell index when they
// fit, else the primitives alone.  The byte field is always read from global memory: one byte
// per lane and link is not worth the LDS (and so the occupancy) it would take.
//
// Voxel broadphase over the primitives: a uniform grid covering every point within `vcap` of
// a primitive.  For each cell, vlist[vstart[c] .. vstart[c+1]) lists every primitive whose
// distance to some point of the cell may be below vcap, as (type << 28 | index, lower bound
// of that distance over the cell), sorted by the bound; the byte field holds the smallest
// bound of the cell, rounded down to multiples of vq (255 = nothing closer than vcap).
struct EnvDev {
    const float4 *rec;
    int32_t off_sph, off_cap, off_cyl, off_box, off_cell, off_vdist, n_rec;
    int32_t n_stage;               // leading records a launch stages in LDS (set per launch)
    int32_t n_sph, n_cap, n_cyl, n_box;
    const int32_t *vstart;         // [n_vox + 1]
    const int2 *vlist;
    int32_t vdim[3], n_vox;
    float vorg[3], vinv, vq, vcap;
    // Uniform grid over a large set of small spheres (point clouds); n_cells == 0 and
    // grid == nullptr when absent.  The cell index is part of the record buffer at off_cell;
    // the rest of the grid is described by *grid.
    const struct GridDev *grid;
    int32_t n_cells;
};

// The point grid and its clearance field, kept in the environment's device buffer (so that a
// walk reads it only where it meets a point cloud).  The points, sorted by cell, stay in global
// memory (L2).
struct GridDev {
    const float4 *pts;             // [n_pts] centre, radius
    // Clearance field of the points on a finer uniform grid: per cell the clearance at the
    // cell's centre, min over points of (distance to the point's centre) - (its radius), in
    // units of pq, rounded down and saturated at 255.  Clearance changes by at most the
    // distance moved, so (value - distance to the centre) bounds it from below anywhere.
    // Locations outside the field are at least 255 pq from every point.
    const uint8_t *pfield;
    int32_t n_pts;
    int32_t gdim[3];
    float gorg[3];
    float ginv;                    // 1 / cell size
    float gmax_r;                  // largest point radius
    int32_t pdim[3];
    float porg[3], pinv, pcell, pq;
};

// Contiguous ranges of the walk's tests that separate waves run for one state: range y is
// [b[y], b[y + 1]), y < n.  The tests are numbered in walk order: step s's environment part is
// number s + blk_first(s) and its self blocks follow it; kAllTests is past every robot's last.
constexpr int kMaxRanges = 32;
constexpr int kAllTests = 1 << 30;
struct StepRanges {
    int32_t n;
    int32_t b[kMaxRanges + 1];
};

// One edge set of a mixed-robot batch.
// Where the endpoints of edge e come from: rows e of qa and qb (pairs == nullptr), or rows
// pairs[2e] and pairs[2e+1] of the node array qa ([n_nodes][dof]).  nst, when not null, gives
// each edge's state count.
struct EdgeSrc {
    const float *qa;
    const float *qb;
    const int32_t *pairs;
    int64_t n_nodes;
    const int32_t *nst;
};

struct BatchSet {
    RobotDev rb;
    EnvDev env;
    int64_t qa_offset;             // float offset of the set's first edge in qa / qb
    int64_t n_edges;
    int64_t out_offset;
    int64_t first;                 // index of the set's first edge in the batch
};

}  // namespace vk
