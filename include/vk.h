/*
 * vk.h -- C ABI of the MI355X vectorized motion-validation library (libvk.so).
 *
 * Implements the hot path of "Motions in Microseconds via Vectorized Sampling-Based Planning"
 * (arXiv 2309.14545): forward kinematics (FK) of a revolute kinematic tree over many
 * configurations at once (Sec. III-B), placement of the robot's collision spheres and
 * sphere-vs-primitive plus self-collision tests (Sec. III-C), and motion (edge) validation by
 * discretising a straight joint-space motion with a "rake" ordering and first-hit early exit
 * (Sec. III-D).  Two extensions use the same kernels: a differentiable squared-penetration
 * cost with a hand-written adjoint, and mixed-robot edge batches replayed from a HIP graph.
 *
 * Conventions shared by every entry point
 *   - Plain C types only.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Batch arrays (q, qa, qb, collide, centres, cost, grad) are DEVICE pointers owned by the
 *     caller; the call only enqueues work on `stream` and returns.  Results are valid once the
 *     caller synchronises that stream.  Description structs are HOST memory, copied at create.
 *   - Handles (vk_robot, vk_env, vk_edge_batch) are owned by the library; destroy them when no
 *     enqueued work still uses them (after a stream sync).
 *   - Configurations in a state batch are structure-of-arrays: q[j * ldq + i] is joint j of
 *     state i (Sec. III-A, struct-of-arrays layout); edge endpoints are array-of-structs:
 *     qa[e * dof + j].
 *   - Output polarity: 1 = in collision (invalid), 0 = free.
 *   - Arguments are checked when the call is made: NULL handles or pointers, n < 0, ld < n and
 *     inconsistent sizes return an error and enqueue nothing; n == 0 is a no-op returning VK_OK.
 *     An asynchronous device fault surfaces as VK_ERR_HIP from a later call or from the
 *     caller's stream synchronisation.  vk_last_error() gives a text for the last error of the
 *     calling thread.
 *   - Joint limits are not checked (validity means collision-free, Sec. III-D).  A state with
 *     a non-finite joint value is reported as colliding; its cost and gradient are NaN.
 *   - A handle may be used from several streams at once; a vk_edge_batch may not.
 *   - Only create, reserve, autotune, release and destroy calls allocate, free or wait.  The
 *     calls that need device scratch take it from the stream's workspace (vk_reserve).
 */
#ifndef VK_H
#define VK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vk_status;
#define VK_OK 0
#define VK_ERR_INVALID_ARG (-1)  /* NULL pointer, negative size, bad index or value          */
#define VK_ERR_SHAPE (-2)        /* leading dimension or size inconsistent with the handle  */
#define VK_ERR_UNSUPPORTED (-3)  /* a description the kernels do not handle (see create)    */
#define VK_ERR_HIP (-4)          /* a HIP runtime call failed                                */
#define VK_ERR_OOM (-5)          /* device allocation failed                                 */

typedef struct vk_robot_s *vk_robot;
typedef struct vk_env_s *vk_env;
typedef struct vk_edge_batch_s *vk_edge_batch;

/*
 * Robot: a kinematic tree of revolute and prismatic joints whose links carry collision spheres
 * (Sec. III-C).  Links are numbered 0..dof; link 0 is the fixed base at the world origin; joint
 * j moves link j+1 and hangs off link parent_link[j] (0 <= parent_link[j] <= j).  Frames follow
 * standard DH (Sec. III-B), with P_j = T_parent(j) * M_j and
 *   revolute:  T_{j+1} = P_j * Rz(q_j + theta_offset_j) Tz(d_j) Tx(a_j) Rx(alpha_j)
 *   prismatic: T_{j+1} = P_j * Rz(theta_offset_j) Tz(d_j + q_j) Tx(a_j) Rx(alpha_j),
 * so joint j turns about, or slides along, the z axis of P_j.  Edge discretisation treats all
 * joint values alike (the resolution is per unit of q: radians or metres).
 */
typedef struct {
    int32_t dof;                  /* 1..64                                                    */
    const int32_t *parent_link;   /* [dof]; NULL = serial chain (parent_link[j] = j)          */
    const float *mount;           /* [dof][12] row-major 3x4 fixed transforms; NULL = identity */
    const float *dh;              /* [dof][5]: a, d, cos(alpha), sin(alpha), theta_offset      */
    const float *q_lo;            /* [dof] informational, not checked; may be NULL             */
    const float *q_hi;            /* [dof] informational, not checked; may be NULL             */
    int32_t n_spheres;            /* S >= 0                                                    */
    const int32_t *sphere_link;   /* [S] link of each sphere, 0..dof, non-decreasing           */
    const float *sphere_xyzr;     /* [S][4] centre in the link frame, radius > 0               */
    int32_t n_self_pairs;         /* P >= 0                                                    */
    const int32_t *self_pairs;    /* [P][2] sphere indices on two different links              */
    const int32_t *joint_type;    /* [dof] 0 revolute, 1 prismatic; NULL = all revolute        */
} vk_robot_desc;

/* Environment of primitives (Sec. III-C: spheres, cylinders, cuboids; capsules = swept
 * spheres).  Counts may be zero (the matching pointer may then be NULL).  A cylinder axis must
 * have unit length and a box rotation must be orthonormal, each within 1e-5 (else
 * VK_ERR_INVALID_ARG). */
typedef struct {
    int32_t n_spheres;   const float *spheres;    /* [n][4]  centre, radius                     */
    int32_t n_capsules;  const float *capsules;   /* [n][7]  end p0, end p1, radius             */
    int32_t n_cylinders; const float *cylinders;  /* [n][8]  centre, unit axis, half height, r  */
    int32_t n_boxes;     const float *boxes;      /* [n][15] centre, row-major 3x3 rotation
                                                   *         (its columns are the box axes),
                                                   *         half extents                       */
} vk_env_desc;

/* Create / destroy a device-resident robot.  The library precomputes, per link, a bounding
 * sphere of the link's spheres (the mid-phase of Sec. III-D) and a bounding capsule (which
 * gates self pairs before the earlier link is posed), and orders the self pairs by their later
 * link so each is tested right after that link is posed (interleaving, Sec. III-D).  Errors: VK_ERR_INVALID_ARG for a bad parent, link index, sphere order, radius
 * <= 0, a pair on one link or a joint type other than 0/1; VK_ERR_UNSUPPORTED for dof > 64. */
vk_status vk_robot_create(const vk_robot_desc *desc, vk_robot *out);
vk_status vk_robot_destroy(vk_robot robot);
int32_t vk_robot_dof(vk_robot robot);
int32_t vk_robot_n_spheres(vk_robot robot);

/*
 * Per-robot specialisation (Sec. III-B: the paper compiles FK and collision checking per robot
 * into straight-line code with the robot's constants folded in).  vk_robot_specialize writes
 * the robot's program (link steps, self-pair blocks and their entries, pose paths, spheres) as
 * constants into a source of the persistent edge kernels, compiles it for the robot's device
 * with the HIP runtime compiler, and loads it; from then on the robot's edge calls
 * (validate_edges, validate_edges_indexed, validate_edges_counted) run these kernels, whose
 * per-step code is unrolled with the constants as instruction operands, instead of the
 * library's kernel that reads the program at run time.  Flags are identical.  A set-up call: it
 * compiles (seconds) unless cache_dir (else NULL) already holds the code object, which it then
 * loads; it stores new code objects there.  vk_robot_use_specialized switches a specialised
 * robot between the two kernels (on = 0: the library's); vk_robot_is_specialized tells which
 * one the robot's calls use (1, 0; -1 for NULL).  vk_robot_spec_source writes the generated
 * source for a description into buf (cap bytes, NUL-terminated, truncated if short) and
 * returns its length including the NUL, or -1 for an invalid description (vk_last_error); it
 * needs no device.  Errors: VK_ERR_HIP when compiling or loading fails (vk_last_error holds the
 * compiler's log), VK_ERR_INVALID_ARG to switch on a robot not specialised.
 */
vk_status vk_robot_specialize(vk_robot robot, const char *cache_dir);
vk_status vk_robot_use_specialized(vk_robot robot, int32_t on);
int32_t vk_robot_is_specialized(vk_robot robot);
int64_t vk_robot_spec_source(const vk_robot_desc *desc, char *buf, int64_t cap);

/* Create / destroy a device-resident environment.  The primitives get a voxel broadphase
 * (per cell, the primitives that may come within 0.5 m, sorted by a distance bound).  A large
 * set of small spheres (more than 1,024, those up to twice the median radius: a point cloud) goes
 * to a uniform grid instead, with a clearance field of 1.5 cm cells (the clearance at each
 * cell's centre, which less the distance to that centre bounds the clearance to the nearest
 * point from below anywhere in the cell; 5.6 MB of device memory in all, 5.2 MB of it the
 * field, for the 20,000 points of a 2.7 m x 2.2 m x 2 m scene).  Queries are unchanged: these structures only skip tests that cannot hit. */
vk_status vk_env_create(const vk_env_desc *desc, vk_env *out);
/* Host-only dry run of vk_env_create (no device needed): checks the description as create
 * does and builds the same structures.  Returns the device bytes the environment would take
 * (-1 for an invalid description, with vk_last_error), and writes the first n_out of: spheres,
 * capsules, cylinders, boxes kept as primitives, spheres moved to the point grid, voxel cells,
 * voxel candidate entries, point-grid cells, clearance-field cells. */
int64_t vk_env_describe(const vk_env_desc *desc, int64_t *out, int32_t n_out);

vk_status vk_env_destroy(vk_env env);

/*
 * Sphere centres of n states (Sec. III-B FK + Sec. III-C, positions only).
 *   q       [dof][ldq] float, device, SoA
 *   centres [S][3][ldc] float, device: centres[(s*3 + axis)*ldc + i]
 * Requires ldq >= n, ldc >= n.
 */
vk_status fk_spheres(vk_robot robot, const float *q, int64_t n, int64_t ldq, float *centres,
                     int64_t ldc, void *stream);

/*
 * Collision flag of n states (Sec. III-C): 1 if some robot sphere overlaps some primitive or
 * some listed self pair overlaps (clearance < 0), else 0.
 *   q       [dof][ldq] float, device, SoA; ldq >= n
 *   collide [n] uint8, device
 * The schedule is the robot's (vk_robot_set_states_split); the two-pass form takes its survivor
 * list from the stream's workspace (vk_reserve with max_states >= n; VK_ERR_SHAPE otherwise).
 */
vk_status validate_states(vk_robot robot, vk_env env, const float *q, int64_t n, int64_t ldq,
                          uint8_t *collide, void *stream);

/*
 * validate_states for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same flags from the same kernels, always
 * in the two-pass schedule (the robot's split, else half of its link steps; a one-step robot
 * runs one pass), with the survivor list in a fixed scratch array compiled into the library
 * (16 MiB + 256 B per GPU, held until the process ends) instead of the stream's workspace.  It
 * needs no vk_reserve and calls no allocating routine.  n may be at most 4,194,304 (2^22),
 * else VK_ERR_SHAPE.  Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (on different streams, or from several threads) race and must be ordered by the
 * caller.  Other errors as validate_states.
 */
vk_status validate_states_noalloc(vk_robot robot, vk_env env, const float *q, int64_t n,
                                  int64_t ldq, uint8_t *collide, void *stream);

/*
 * Collision flag of n_edges straight joint-space motions (Sec. III-D).  Edge e from qa to qb is
 * discretised into n_e states q_k = qa + k/(n_e-1) (qb - qa), k = 0..n_e-1, both endpoints
 * included, with n_e = n_states[e] if n_states is given, else
 *   n_e = max(2, ceil(max_j |qb_j - qa_j| / resolution) + 1)
 * evaluated in double precision (so it is exact for FP32 inputs and a power-of-two
 * resolution).  collide[e] = OR of the state flags.  States are visited in rake order (lane l
 * of a 64-wide wavefront takes states l*ceil(n_e/64) + k at step k) and the edge stops at the
 * first colliding state found; the flag does not depend on the order.  All edges run in one
 * persistent launch that pulls edges from a device work queue.
 *   qa, qb    [n_edges][dof] float, device
 *   n_states  [n_edges] int32, device, each >= 2; or NULL
 *   resolution > 0 (radians per step, per joint); ignored when n_states is given
 *   collide   [n_edges] uint8, device
 * An edge of more than 2^24 states (an explicit count, or a computed one, which saturates at
 * 2^31 - 1 for endpoints very far apart) is not validated: its flag is 1.  The launch takes its
 * work-queue counters from the stream's workspace (vk_reserve; VK_ERR_SHAPE without one) and
 * its shape from the robot's launch settings (vk_robot_set_edge_launch).
 */
vk_status validate_edges(vk_robot robot, vk_env env, const float *qa, const float *qb,
                         const int32_t *n_states, int64_t n_edges, float resolution,
                         uint8_t *collide, void *stream);

/* The state count validate_edges gives the edge qa -> qb (host arrays [dof]) at `resolution`:
 * max(2, ceil(max_j |qb_j - qa_j| / resolution) + 1) in double precision, saturated at
 * 2^31 - 1.  Returns -1 for NULL arrays, dof outside [1, 64], a non-finite endpoint (such an
 * edge is reported as colliding) or a resolution that is not finite and > 0. */
int64_t vk_edge_states(const float *qa, const float *qb, int32_t dof, float resolution);

/* Same contract as validate_edges, but one kernel launch per edge (the plain baseline the
 * batched launch is measured against). */
vk_status validate_edges_per_edge(vk_robot robot, vk_env env, const float *qa, const float *qb,
                                  const int32_t *n_states, int64_t n_edges, float resolution,
                                  uint8_t *collide, void *stream);

/* Edge validation with endpoints given by index: edge e runs from node pairs[2e] to node
 * pairs[2e+1] of `nodes` (device, AoS [n_nodes][dof]); otherwise exactly validate_edges (same
 * discretisation, rake and early exit, same kernel).  This is the form a PRM roadmap or a batch
 * of shortcut candidates takes (Sec. III-E: the planners built on the edge validator).  A pair
 * with a negative entry is a hole: no edge, flag 0 (vk_knn_pairs writes (-1, -1) for
 * duplicates).  An index >= n_nodes makes the edge's flag 1.  pairs: device int32 [n_edges][2].
 * Errors as validate_edges. */
vk_status validate_edges_indexed(vk_robot robot, vk_env env, const float *nodes, int64_t n_nodes,
                                 const int32_t *pairs, const int32_t *n_states, int64_t n_edges,
                                 float resolution, uint8_t *collide, void *stream);

/* k nearest neighbours of each of n samples (device, AoS [n][dim]) among the others, by the
 * Euclidean norm of the configuration difference (the roadmap neighbourhoods of a PRM,
 * Sec. III-E).  Writes idx [n][k] (int32) and dist2 [n][k] (FP32 squared distances), each row
 * ascending.  The squared distance is accumulated in dimension order with separately rounded
 * FP32 products and sums (no fused multiply-add); equal distances go to the lower index.
 * Samples at a non-finite distance are skipped; a row with fewer than k neighbours ends in
 * index -1 and distance +inf.  1 <= dim <= 64, 1 <= k <= 32 (else VK_ERR_UNSUPPORTED /
 * VK_ERR_INVALID_ARG).  Brute force: O(n^2 dim) work, meant for roadmaps of up to ~10^5
 * samples.  The partial lists live in the stream's workspace (vk_reserve with max_knn_samples
 * >= n and max_knn_k >= k; VK_ERR_SHAPE otherwise). */
vk_status vk_knn(const float *x, int64_t n, int32_t dim, int32_t k, int32_t *idx, float *dist2,
                 void *stream);

/* Undirected roadmap edges from kNN lists (device idx [n][k]): slot i*k+m of pairs ([n*k][2],
 * device int32) holds (i, j) for j = idx[i][m] when i < j or when i is not in j's list, else
 * the hole (-1, -1), so each undirected edge is listed once, at a fixed slot.  Entries outside
 * [0, n) or equal to i become holes. */
vk_status vk_knn_pairs(const int32_t *idx, int64_t n, int32_t k, int32_t *pairs, void *stream);

/*
 * Tree primitives of a many-query RRT-Connect (the planner of Sec. III-E, run for nq queries
 * in lockstep; the host loop lives in the Python package).  Query q owns a tree of up to `cap`
 * nodes: nodes[q][cap][dof] (device FP32), parents[q][cap] (int32), sizes[q] (int32, nodes in
 * use).  All arrays are device memory; per-query vectors are [nq] or [nq][dof].
 *
 * vk_tree_nearest: near[q] = index of the tree node nearest to targets[q] (Euclidean; squared
 *   distance accumulated in joint order with separately rounded FP32 products and sums, ties to
 *   the lower index), or -1 for an empty tree or when active (optional, uint8 [nq]) is 0.
 * vk_tree_steer: qnew[q] = targets[q] if it lies within `step` of node near[q] (reached[q] = 1),
 *   else near + (targets - near) * step / |targets - near| (reached[q] = 0); near < 0 copies the
 *   target with reached = 0.  step must be finite and > 0.
 * vk_tree_append: where ok[q] != 0, near[q] is a node of the tree and the tree has room,
 *   appends qnew[q] with parent near[q] and writes its index to added[q]; else added[q] = -1.
 * Errors: VK_ERR_INVALID_ARG for NULL arrays, cap < 1, dof outside [1, 64] or nq < 0.
 */
vk_status vk_tree_nearest(const float *nodes, const int32_t *sizes, int32_t cap, int32_t dof,
                          int64_t nq, const float *targets, const uint8_t *active, int32_t *near,
                          void *stream);
vk_status vk_tree_steer(const float *nodes, int32_t cap, int32_t dof, int64_t nq,
                        const int32_t *near, const float *targets, float step, float *qnew,
                        uint8_t *reached, void *stream);
vk_status vk_tree_append(float *nodes, int32_t *parents, int32_t *sizes, int32_t cap, int32_t dof,
                         int64_t nq, const float *qnew, const int32_t *near, const uint8_t *ok,
                         int32_t *added, void *stream);

/* Fused steps of the many-query RRT-Connect (the planner of Sec. III-E run for nq queries in
 * lockstep), so that one extension of every query's tree is three launches: vk_rrt_extend,
 * validate_edges on its edges, vk_rrt_commit.  Arrays as for the tree primitives above (device,
 * caller-owned, row-major): nodes [nq][cap][dof], sizes and parents per tree, targets, qnear and
 * qnew [nq][dof].
 *
 * vk_rrt_extend: for each query with active[q] != 0 (uint8 [nq], required), near[q] = the tree
 *   node nearest to targets[q] as vk_tree_nearest finds it, and qnew[q], reached[q] as
 *   vk_tree_steer computes them from it (bit-identical); qnear[q] = that node, so that
 *   qnear -> qnew is the edge to check.  An inactive query, or one whose tree is empty, gets
 *   near = -1, reached = 0 and qnear = qnew = the tree's first node (the target for an empty
 *   tree): a zero-length edge.  step must be finite and > 0.
 * vk_rrt_commit: after validate_edges(qnear, qnew) -> flags (uint8 [nq], 1 = collides), for each
 *   query with going[q] != 0: adds 1 to *edges (one device uint64, not cleared) and appends
 *   qnew[q] with parent near[q] when flags[q] == 0, near[q] is a node and the tree has room;
 *   added[q] = the new node's index, else -1 (also for queries not going).  going (uint8 [nq])
 *   is updated in place.  With from_added == NULL (an extension toward a sample):
 *   going[q] = (added[q] >= 0).  Otherwise (an extension toward the node from_added[q] that the
 *   other tree just added): a node added with reached[q] != 0 joins the trees, so solved[q] = 1,
 *   meet_this[q] = added[q] and meet_from[q] = from_added[q] (int64 [nq] each, this tree's and
 *   the other tree's meeting nodes); going[q] = (added[q] >= 0 && reached[q] == 0).  Entries of
 *   queries that do not meet are left as they are.
 * Errors: VK_ERR_INVALID_ARG for NULL arrays (meet_this, meet_from and solved may be NULL only
 *   without from_added), cap < 1, dof outside [1, 64] or nq < 0. */
vk_status vk_rrt_extend(const float *nodes, const int32_t *sizes, int32_t cap, int32_t dof,
                        int64_t nq, const float *targets, const uint8_t *active, float step,
                        float *qnear, float *qnew, int32_t *near, uint8_t *reached, void *stream);
vk_status vk_rrt_commit(float *nodes, int32_t *parents, int32_t *sizes, int32_t cap, int32_t dof,
                        int64_t nq, const float *qnew, const int32_t *near, const uint8_t *reached,
                        const uint8_t *flags, uint8_t *going, int32_t *added,
                        const int32_t *from_added, int64_t *meet_this, int64_t *meet_from,
                        uint8_t *solved, uint64_t *edges, void *stream);

/*
 * Randomized shortcutting of many paths at once (the path simplification of Sec. III-E, run as
 * rounds over n_paths paths): a round is vk_shortcut_propose, validate_edges_indexed on its
 * pairs with `paths` as the node array, then vk_shortcut_apply.  Paths are device FP32
 * [n_paths][max_len][dof] (waypoint w of path p is node p * max_len + w); lens [n_paths] (int32)
 * holds the waypoints in use.  Every removed stretch of waypoints is replaced by a straight
 * edge that validate_edges found free, so a path stays valid and its length does not grow.
 *
 * vk_shortcut_propose: k candidates per path, pairs [n_paths * k][2] (int32 node indices), from
 *   the caller's random words rnd [n_paths * k][2] (uint32): i = rnd0 mod (len - 2),
 *   j = i + 2 + rnd1 mod (len - i - 2), so 0 <= i, i + 2 <= j <= len - 1.  A path with fewer
 *   than 3 waypoints gets holes (-1, -1).
 * vk_shortcut_apply: per path, among its candidates with collide == 0 (the flags of the
 *   validate_edges_indexed call on those pairs), the one with the largest j - i (ties to the
 *   lower candidate index) is spliced in: waypoints i+1 .. j-1 are removed, the rest move down
 *   and lens shrinks.  accepted [n_paths] (uint8, optional) is 1 where a shortcut was taken.
 * Errors: VK_ERR_INVALID_ARG for NULL arrays, n_paths < 0, max_len < 1, k outside [1, 64] or
 * dof outside [1, 64]; VK_ERR_SHAPE when n_paths * max_len reaches 2^31.
 */
vk_status vk_shortcut_propose(const int32_t *lens, int64_t n_paths, int32_t max_len, int32_t k,
                              const uint32_t *rnd, int32_t *pairs, void *stream);
vk_status vk_shortcut_apply(float *paths, int32_t *lens, int64_t n_paths, int32_t max_len,
                            int32_t dof, int32_t k, const int32_t *pairs, const uint8_t *collide,
                            uint8_t *accepted, void *stream);

/* Measurement variant of validate_edges: the same flags from the same kernel code, which in
 * addition adds to flops[0..7] (eight device uint64, not cleared by the call) the FP32
 * operations the launch executed, by the model's count per operation (fused multiply-add = 2;
 * revolute joint 30, mount 63, sphere placement 18, sphere-sphere and self pair 11, capsule 25,
 * box 34, cylinder 35; self-block gates: capsule bound against capsule bound 67, sphere bound
 * against capsule bound 28, placing a capsule half-vector 15; a point-cloud clearance lookup
 * 23), summed over the lanes that execute it.  flops[0] is the total.  flops[1..4] are the
 * method's own work: FK and sphere placement, culling (voxel lookups and link bounding-sphere
 * tests), fine environment tests, and self pairs (their gates and tests).  flops[5..6] are work
 * the implementation adds: re-posing (an earlier link posed again for a self block, a tree
 * branch rebuilt from the base, the earlier link's spheres placed again), and everything the
 * surplus rake lanes execute (an edge of n states leaves 64 * ceil(n / 64) - n lanes of its
 * rake over; they repeat the last state).  flops[7] counts rake slots of real states walked
 * (one per lane and rake step up to the step that ends the edge), which the rake schedule and
 * the first hit alone decide.  Early exits, skipped tests and lanes masked off by divergent
 * control flow add nothing. */
vk_status validate_edges_counted(vk_robot robot, vk_env env, const float *qa, const float *qb,
                                 const int32_t *n_states, int64_t n_edges, float resolution,
                                 uint8_t *collide, uint64_t *flops, void *stream);

/*
 * Squared-penetration cost per state (differentiable extension):
 *   cost = sum_{s,o} max(0, r_s - sd_o(c_s))^2 + sum_{(s,t) in pairs} max(0, r_s + r_t - |c_s - c_t|)^2
 * over every robot sphere s and primitive o (sd = signed distance) and every listed self pair.
 *   q [dof][ldq] float, device; cost [n] float, device
 */
vk_status penetration_cost_fwd(vk_robot robot, vk_env env, const float *q, int64_t n,
                               int64_t ldq, float *cost, void *stream);

/*
 * Adjoint of penetration_cost_fwd: grad_q[j][i] = grad_cost[i] * d cost_i / d q_j.  The kernel
 * recomputes FK, forms the force f_s = d cost / d c_s on every sphere and pulls it back through
 * the joint axes (dq_j = z_j . sum over spheres beyond j of (c_s - o_j) x f_s).
 *   grad_cost [n] float, device; grad_q [dof][ldg] float, device, ldg >= n
 */
vk_status penetration_cost_bwd(vk_robot robot, vk_env env, const float *q, int64_t n,
                               int64_t ldq, const float *grad_cost, float *grad_q, int64_t ldg,
                               void *stream);

/*
 * The cost and its gradient from one adjoint walk (the adjoint computes the cost anyway):
 * cost [n] exactly as penetration_cost_fwd gives it, and grad_q[j][i] = d cost_i / d q_j as
 * penetration_cost_bwd gives it for grad_cost = 1.  One launch instead of two for a forward and
 * backward pass (the autograd function calls this in its forward when q needs a gradient and
 * scales the result by grad_cost in its backward).  Arguments and errors as the two calls.
 */
vk_status penetration_cost_fwd_grad(vk_robot robot, vk_env env, const float *q, int64_t n,
                                    int64_t ldq, float *cost, float *grad_q, int64_t ldg,
                                    void *stream);

/*
 * Mixed-robot edge batches: several edge sets, each with its own robot and environment, run as
 * one persistent launch, held in a HIP graph {work-queue reset -> launch} built at create and
 * replayed by vk_edge_batch_run.  Set k covers edges [qa_offset / dof_k, ... + n_edges) of the
 * qa/qb arrays passed to run (AoS with that set's robot dof, offsets in floats) and writes
 * collide[out_offset + i].  run takes the device arrays of each replay (the graph's launch is
 * re-pointed when they change, without rebuilding it); they must hold every set's edges and
 * flags.  The launch shape is fixed at create: block_threads and blocks_per_cu as for
 * vk_robot_set_edge_launch, both 0 for the default (256, 4).  A batch owns one set of
 * work-queue counters, so replays of one batch must not overlap in time: replays on one stream
 * are ordered by it, replays on different streams must be ordered by the caller (events).
 * Different batches are independent.  Create allocates (device memory for the set records and
 * counters); run does not.
 */
typedef struct {
    int32_t robot;          /* index into robots[] */
    int32_t env;            /* index into envs[]   */
    int64_t qa_offset;      /* float offset of the set's first edge in qa and qb */
    int64_t n_edges;
    int64_t out_offset;     /* offset of the set's first flag in collide */
} vk_edge_set;

vk_status vk_edge_batch_create(const vk_robot *robots, int32_t n_robots, const vk_env *envs,
                               int32_t n_envs, const vk_edge_set *sets, int32_t n_sets,
                               float resolution, int32_t block_threads, int32_t blocks_per_cu,
                               vk_edge_batch *out);
vk_status vk_edge_batch_run(vk_edge_batch batch, const float *qa, const float *qb,
                            uint8_t *collide, void *stream);
vk_status vk_edge_batch_get_launch(vk_edge_batch batch, int32_t *block_threads,
                                   int32_t *blocks_per_cu);
vk_status vk_edge_batch_destroy(vk_edge_batch batch);

/*
 * Workspace.  The persistent edge launches need work-queue counters (33 slots of 32 KiB: a launch
 * takes the next slot of a ring that one small launch zeroes whenever it wraps), two-pass
 * validate_states a survivor list (4 bytes per state) and vk_knn partial lists; they take them
 * from a workspace the library keeps per (device, stream).  vk_reserve creates it for `stream`
 * on the current device, or grows it to cover calls of up to max_states states (two-pass
 * validate_states) and up to max_knn_samples samples with k <= max_knn_k (vk_knn); 0 sizes
 * reserve the counters only.  It never shrinks, and a grown workspace keeps its earlier buffers
 * until vk_release (a graph captured on the stream may still point at them).  vk_reserve may
 * allocate, so it is a set-up call: made while the stream is being captured it fails with
 * VK_ERR_SHAPE if the workspace would have to grow, and does nothing otherwise.  The calls
 * that use the workspace never allocate, free or wait: they return VK_ERR_SHAPE when their
 * stream has no workspace or too small a one.  vk_release waits for the stream, then frees its
 * workspace (graphs captured on it must not be replayed afterwards).  Errors:
 * VK_ERR_INVALID_ARG for negative sizes or max_knn_k > 32, VK_ERR_OOM.
 */
vk_status vk_reserve(void *stream, int64_t max_states, int64_t max_knn_samples, int32_t max_knn_k);
/*
 * Workspace for the adjoint of the squared-penetration cost over the sphere model (Sec. III-C;
 * penetration_cost_bwd, penetration_cost_fwd_grad) on `stream`, for up to max_states states of
 * this robot.  The adjoint keeps per-link force and moment slots for
 * every state (24 bytes per link); in LDS they hold it to a few waves per CU, so a batch that
 * needs more than one round of those waves keeps them in this workspace instead and runs at
 * four waves per SIMD (262,144 7-DoF states: 175 -> 148 us).  For sizes whose slots stay in LDS
 * nothing beyond the queue counters is reserved.  Without the workspace the calls keep the slots
 * in LDS: the results are the same either way.  A set-up call like vk_reserve (it allocates, and
 * fails with VK_ERR_SHAPE on a stream under capture when the workspace would grow).  Errors:
 * VK_ERR_INVALID_ARG for a NULL robot or max_states < 0, VK_ERR_SHAPE above 2^31 - 1 states.
 */
vk_status vk_reserve_cost(void *stream, vk_robot robot, int64_t max_states);

vk_status vk_release(void *stream);

/*
 * Launch settings, kept per robot handle.
 * Edge launches of the robot (validate_edges, validate_edges_indexed, validate_edges_counted):
 * workgroup size block_threads (a multiple of 64 up to 1024), workgroups per compute unit
 * blocks_per_cu (1..64), and tickets_per_wave (1..64): about that many work-queue tickets per
 * wave, which sets how many edges one ticket hands out.  All three 0 restore the defaults
 * (256, 4, 8).  A launch whose per-wave LDS cache (3 floats per lane for each link step a later
 * self pair reads, 2 more with the capsule halves, and optionally 2 per joint) would not fit
 * uses the largest smaller workgroup that fits.
 * States (validate_states): with num > 0 it runs in two passes.  Pass 1 tests the first
 * floor(S * num / den) of the robot's S link steps for every state; pass 2 walks only the
 * states still free, packed densely into waves, testing the remaining steps.  Flags are
 * identical to one pass; the split pays off when most states collide early (a wave of
 * independent states walks as long as its last live lane), and costs time when they do not.
 * (0, 1) = one pass, the default.  The two-pass form needs a workspace (vk_reserve).
 * Invalid values: VK_ERR_INVALID_ARG.  Settings may change between calls; a call uses the
 * values it reads when it is made.
 */
/*
 * Waves sharing one edge (long edges: the rake of Sec. III-D spread over several 64-lane
 * waves).  With parts P > 1 every edge becomes P work items; part p walks the rake steps
 * p, p + P, p + 2P, ... of the edge (each part starts with a step that samples the whole
 * motion), a part that finds a collision sets the edge's flag, and the others stop before
 * their next step.  Flags are those of P = 1.  An edge of n states has ceil(n / 64) rake steps,
 * so parts pay off when that is well above P (fine resolutions, long explicit counts); for
 * short edges the extra items only cost queue tickets.  1..64 (else VK_ERR_INVALID_ARG),
 * default 1; vk_robot_get_edge_parts returns it (-1 for NULL).
 */
vk_status vk_robot_set_edge_parts(vk_robot robot, int32_t parts);
int32_t vk_robot_get_edge_parts(vk_robot robot);

/*
 * Test ranges of a small edge batch (validate_edges, validate_edges_indexed).  A batch of a few
 * dozen one-wave items (edges times their rake parts) is bound by the latency of one wave's walk
 * (Sec. III-D: the whole rake of an edge walks every test in every state).  Each edge's walk is then split over up to max_ranges ranges of its tests (in walk
 * order: each link step's environment part, then that step's self-pair blocks; ranges of equal
 * test count), each run by its own waves over the edge's whole rake (posing the earlier steps),
 * and an edge's flag is 1 when any range finds a collision: the flags of the unsplit walk.
 * -1 (the default) splits only batches of at most one wave per two compute units, into about
 * one wave per two compute units in all (at most one range per test and 32); 0 or 1 never
 * splits; 2..32 splits into at
 * most that many ranges at any batch size.  validate_edges_counted never splits.  Errors:
 * VK_ERR_INVALID_ARG outside [-1, 32].  vk_robot_get_edge_ranges returns the setting (-2 for
 * NULL).
 */
vk_status vk_robot_set_edge_ranges(vk_robot robot, int32_t max_ranges);
int32_t vk_robot_get_edge_ranges(vk_robot robot);
vk_status vk_robot_set_edge_launch(vk_robot robot, int32_t block_threads, int32_t blocks_per_cu,
                                   int32_t tickets_per_wave);
vk_status vk_robot_get_edge_launch(vk_robot robot, int32_t *block_threads, int32_t *blocks_per_cu,
                                   int32_t *tickets_per_wave);
vk_status vk_robot_set_states_split(vk_robot robot, int32_t num, int32_t den);
vk_status vk_robot_get_states_split(vk_robot robot, int32_t *num, int32_t *den);

/*
 * Test ranges of a small validate_states batch (one pass only).  A batch of fewer than eight waves
 * (64 states each) per compute unit leaves the chip short of waves and is bound by the latency
 * of one wave's walk.  Each state's walk is then split over up to max_ranges contiguous ranges of
 * its tests (in walk order: each link step's environment part, then each of that step's
 * self-pair blocks), each run by its own waves (posing the earlier steps, running its own
 * tests), and a state's flag is 1 when any range finds a collision: the same flags as the whole
 * walk.  -1 (the default) picks the count for the batch (about equal work per range, at most
 * one per test and 32 in all, and no more than keep the split batch within 16 waves per CU);
 * 0 or 1 never splits; 2..32 splits into at most that many ranges at any batch size.  Errors:
 * VK_ERR_INVALID_ARG outside [-1, 32].
 */
vk_status vk_robot_set_states_ranges(vk_robot robot, int32_t max_ranges);
vk_status vk_robot_get_states_ranges(vk_robot robot, int32_t *max_ranges);

/*
 * Autotuner (a set-up call: it allocates, launches and waits for `stream`).  vk_autotune_edges
 * times validate_edges on the given batch (same arguments) for every workgroup size in
 * {64, 128, 256, 512, 1024}, workgroups per CU in {1, 2, 4, 8} (at most 2,048 threads per CU)
 * and tickets per wave in {4, 8, 16}, each the median of 7 launches after one untimed launch,
 * times the four fastest again in three interleaved rounds (each scored by the median of its
 * rounds), then parts per edge in {1, 2, 4, 8} at the winner, and sets the fastest on the
 * robot.  vk_autotune_states does the same for the validate_states
 * schedules one pass, and two passes split after 1/3, 1/2 and 2/3 of the steps.  With a
 * cache_path (else NULL), results are kept in that JSON file keyed by the workload's class
 * (device, dof, sphere count, primitive count and batch size, the counts rounded up to powers of
 * two): a class already in the file is applied without timing unless force != 0.  Both reserve
 * the stream's workspace they need.  Errors as the timed call.
 */
vk_status vk_autotune_edges(vk_robot robot, vk_env env, const float *qa, const float *qb,
                            const int32_t *n_states, int64_t n_edges, float resolution,
                            const char *cache_path, int32_t force, void *stream);
vk_status vk_autotune_states(vk_robot robot, vk_env env, const float *q, int64_t n, int64_t ldq,
                             const char *cache_path, int32_t force, void *stream);

/* Text of the calling thread's last non-OK status ("" if none). */
const char *vk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VK_H */
