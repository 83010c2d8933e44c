// Kernel launchers shared between the kernel translation unit and the C-ABI layer.  The
// EnvDev passed to a launcher carries in n_stage the number of leading records to stage in LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "vk_types.hpp"

namespace vk {

hipError_t launch_fk_spheres(const RobotDev &rb, const float *q, int64_t n, int64_t ldq,
                             float *out, int64_t ldc, hipStream_t s);
// State validation; with split > 0 and scratch (states_scratch_bytes(n) bytes) it runs in two
// passes, the second over the states still free after the walk's tests before number `split`
// (tests numbered as for StepRanges).  Without the two passes, `ranges` (optional, n > 1)
// splits a small batch's walk over test ranges run by separate waves.
// states_split gives the link step where the first pass ends (0: one pass); the caller turns
// it into that step's first test number.
int states_split(const RobotDev &rb, int64_t n, int num, int den);
size_t states_scratch_bytes(int64_t n);
hipError_t launch_validate_states(const RobotDev &rb, const EnvDev &ed, const float *q, int64_t n,
                                  int64_t ldq, uint8_t *out, int split, void *scratch,
                                  hipStream_t s, const StepRanges *ranges = nullptr);
// The allocation-free form's scratch (a file-scope device array, states_scratch_bytes of up to
// noalloc_max_states() states): its address on the current device, looked up once per device.
int64_t noalloc_max_states();
hipError_t noalloc_scratch(void **ptr);
// Zero the work-queue counters, and with `flags` also n_flags flags (one launch).
hipError_t launch_reset_queue(unsigned long long *queue, hipStream_t s, uint8_t *flags = nullptr,
                              int64_t n_flags = 0);
hipError_t launch_shortcut_propose(const int32_t *lens, int64_t P, int M, int K,
                                  const uint32_t *rnd, int32_t *pairs, hipStream_t s);
hipError_t launch_shortcut_apply(float *paths, int32_t *lens, int64_t P, int M, int dof, int K,
                                const int32_t *pairs, const uint8_t *flags, uint8_t *accepted,
                                hipStream_t s);
hipError_t launch_validate_edges(const RobotDev &rb, const EnvDev &ed, const EdgeSrc &src,
                                 int64_t n_edges, float res, uint8_t *out,
                                 unsigned long long *queue, int grid, int block, int tickets,
                                 int parts, int tparts, hipStream_t s,
                                 unsigned long long *flops = nullptr);
// The walk's headers, embedded in the library for the runtime compiler (generated at build time).
const char *const *embedded_header_names(int *n);
const char *const *embedded_header_texts();
// The persistent edge kernels compiled for one robot (vk_robot_specialize), by staging mode;
// `counted` are the instrumented variants.
struct SpecEdgeKernels {
    hipFunction_t edges[3] = {nullptr, nullptr, nullptr};
    hipFunction_t counted[3] = {nullptr, nullptr, nullptr};
};
hipError_t launch_validate_edges_spec(const SpecEdgeKernels &K, const RobotDev &rb, const EnvDev &ed,
                                      const EdgeSrc &src, int64_t n_edges, float res, uint8_t *out,
                                      unsigned long long *queue, int grid, int block, int tickets,
                                      int parts, int tparts, hipStream_t s,
                                      unsigned long long *flops = nullptr);
hipError_t launch_validate_edge_one(const RobotDev &rb, const EnvDev &ed, const EdgeSrc &src,
                                    int64_t e, float res, uint8_t *out, hipStream_t s);
// kNN runs as partial lists over candidate parts plus a merge; the partial lists need a
// workspace of knn_workspace_bytes(n, k) bytes.
int knn_parts(int64_t n);
size_t knn_workspace_bytes(int64_t n, int k);
// An upper bound of knn_workspace_bytes(n, k) over every n <= max_n (the part count falls as n
// grows, so the bytes are not monotone in n).
size_t knn_workspace_bound(int64_t max_n, int k);
hipError_t launch_knn(const float *x, int64_t n, int dim, int k, int32_t *idx, float *d2,
                      void *workspace, hipStream_t s);
hipError_t launch_knn_pairs(const int32_t *idx, int64_t n, int k, int32_t *pairs, hipStream_t s);
hipError_t launch_tree_nearest(const float *nodes, const int32_t *sizes, int cap, int dof,
                               int64_t nq, const float *targets, const uint8_t *active,
                               int32_t *near, hipStream_t s);
hipError_t launch_tree_steer(const float *nodes, int cap, int dof, int64_t nq, const int32_t *near,
                             const float *targets, float step, float *qnew, uint8_t *reached,
                             hipStream_t s);
hipError_t launch_tree_append(float *nodes, int32_t *parents, int32_t *sizes, int cap, int dof,
                              int64_t nq, const float *qnew, const int32_t *near,
                              const uint8_t *ok, int32_t *added, hipStream_t s);
hipError_t launch_rrt_extend(const float *nodes, const int32_t *sizes, int cap, int dof,
                             int64_t nq, const float *targets, const uint8_t *active, float step,
                             float *qnear, float *qnew, int32_t *near, uint8_t *reached,
                             hipStream_t s);
hipError_t launch_rrt_commit(float *nodes, int32_t *parents, int32_t *sizes, int cap, int dof,
                             int64_t nq, const float *qnew, const int32_t *near,
                             const uint8_t *reached, const uint8_t *flags, uint8_t *going,
                             int32_t *added, const int32_t *from_added, int64_t *meet_this,
                             int64_t *meet_from, uint8_t *solved, uint64_t *edges,
                             hipStream_t s);
hipError_t launch_cost_fwd(const RobotDev &rb, const EnvDev &ed, const float *q,
                           int64_t n, int64_t ldq, float *cost, hipStream_t s);
size_t cost_bwd_slot_bytes(const RobotDev &rb, int block, int cf);
// Per-workgroup LDS of the walk caches (link bound centres and joint sines/cosines, per wave).
// With jc the joint sine/cosine slots are included; launchers add them only when they cost no
// resident workgroups, so callers size their checks without them.
size_t walk_lds_bytes(const RobotDev &rb, int block, int cf = 0);
// Workgroup size of the state and cost-forward launches: `want` threads, fewer (whole waves,
// at least one) when the per-wave walk caches of a long robot would not fit the LDS.
int walk_block(const RobotDev &rb, int want);
// The adjoint: grad = gcost * d cost / d q (gcost NULL: the plain gradient); with `cost` the
// per-state cost is stored too.  With gslots (cost_bwd_global_slot_bytes(rb, n, block) bytes)
// the per-link force slots go to that global scratch instead of the LDS.
hipError_t launch_cost_bwd(const RobotDev &rb, const EnvDev &ed, const float *q,
                           int64_t n, int64_t ldq, const float *gcost, float *grad, int64_t ldg,
                           int block, hipStream_t s, float *cost = nullptr,
                           float *gslots = nullptr);
size_t cost_bwd_global_slot_bytes(const RobotDev &rb, int64_t n, int block);
// Resident waves per CU of the adjoint with its slots in LDS (workgroups of `block` threads).
int cost_bwd_lds_waves_per_cu(const RobotDev &rb, int block);

// A kernel launch spelled out for a graph node: the kernel, its shape and its argument values
// (args[i] points at the i-th value held in the node itself, so a node must not be copied
// after it is filled).
struct KernelNode {
    const void *fn = nullptr;
    dim3 grid, block;
    size_t shmem = 0;
    struct {
        unsigned long long *p;
        unsigned long long v;
        int n, stride;
    } fill{};
    struct {                        // k_validate_edge_batch's arguments, in order
        const BatchSet *sets;
        const int32_t *edge_set;
        int n_sets;
        int64_t total;
        float res;
        const float *qa, *qb;
        uint8_t *out;
        unsigned long long *queue;
        int chunk, floats, cf;
    } batch{};
    void *args[12] = {};
};
// The queue reset of a persistent launch as a node: writes v to n counters `stride` words apart.
void fill_node(KernelNode &L, unsigned long long *p, unsigned long long v, int n, int stride);
// The mixed-robot persistent launch as a node; the caller sets batch.qa, .qb and .out.
void edge_batch_node(KernelNode &L, const BatchSet *sets, const int32_t *edge_set, int n_sets,
                     int64_t total, float res, unsigned long long *queue, int grid, int block,
                     int tickets, int max_slots, int max_dof);

}  // namespace vk
