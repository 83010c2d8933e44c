// C-ABI layer of libvk: handle creation (robot program, environment records, point-cloud grid),
// argument checks and kernel launches.  No exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include <unistd.h>

#include "vk.h"
#include "vk_launch.hpp"
#include "vk_types.hpp"

using namespace vk;

namespace {

thread_local std::string g_err;

struct VkError : std::runtime_error {
    vk_status code;
    VkError(vk_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void raise(vk_status c, const std::string &m) { throw VkError(c, m); }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) raise(VK_ERR_OOM, std::string(what) + ": out of device memory");
    raise(VK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
vk_status guarded(F &&f) {
    try {
        f();
        return VK_OK;
    } catch (const VkError &e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return VK_ERR_OOM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return VK_ERR_INVALID_ARG;
    }
}

struct DeviceInfo {
    int n_cu = 0;
    size_t max_lds = 0;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;

const DeviceInfo &device_info(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) return it->second;
    DeviceInfo d;
    int v = 0;
    hip_check(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev), "device CUs");
    d.n_cu = v;
    hip_check(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
              "device LDS");
    d.max_lds = (size_t)v;
    return g_dev[dev] = d;
}

int current_device() {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    return dev;
}

// Workspace of one (device, stream): the persistent launches' work-queue counters and the
// scratch of the multi-kernel calls (the survivor list of two-pass state validation, kNN's
// partial lists).  Calls on one stream are ordered, so they share it.  Only vk_reserve
// allocates it; a grown workspace keeps its earlier buffers alive (a graph captured on the
// stream may still point at them) until vk_release.
// The queue counters come in kQueueRing + 1 slots of kQueueBytes.  The first kQueueRing are
// handed out in turn, one per edge launch, and all zeroed by one small launch when the ring
// wraps, so most launches need no reset of their own.  The last slot is zeroed by the launch
// that takes it: edges split over several waves (their flags are zeroed with it) and launches
// on a stream being captured into a graph (every replay of the graph must start from zero).
constexpr int kQueueRing = 32;
constexpr size_t kQueueSlotWords = (size_t)kQueues * kQueueWords;
struct Workspace {
    unsigned long long *queue = nullptr;
    int next_slot = kQueueRing;            // the ring's next clean slot; kQueueRing: all used
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    std::vector<void *> retired;
};
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// The workspace of the current device and stream `s`, with at least `scratch_bytes` of scratch;
// the hot calls never allocate, so a missing or smaller one is an error naming vk_reserve.
const Workspace &workspace_for(hipStream_t s, size_t scratch_bytes, const char *what) {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find(std::make_pair(dev, s));
    if (it == g_ws.end())
        raise(VK_ERR_SHAPE, std::string(what) + ": no workspace for this stream (call vk_reserve first)");
    if (it->second.scratch_bytes < scratch_bytes)
        raise(VK_ERR_SHAPE, std::string(what) + ": the stream's workspace holds " +
                                std::to_string(it->second.scratch_bytes) + " scratch bytes, the call needs " +
                                std::to_string(scratch_bytes) + " (call vk_reserve with larger sizes)");
    return it->second;
}

// Scratch bytes that calls of up to these sizes need.
size_t reserve_bytes(int64_t max_states, int64_t max_knn_n, int max_knn_k) {
    size_t b = max_states > 0 ? states_scratch_bytes(max_states) : 0;
    if (max_knn_n > 0 && max_knn_k > 0) b = std::max(b, knn_workspace_bound(max_knn_n, max_knn_k));
    return b;
}

// Launch settings kept per robot handle (the autotuner sets them per workload).
constexpr int kDefaultEdgeBlock = 256, kDefaultEdgeBpc = 4, kDefaultTickets = 8;

// Device blob: several host arrays copied into one allocation at 256-byte aligned offsets.
struct Blob {
    std::vector<char> host;
    size_t add(const void *p, size_t bytes) {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + std::max<size_t>(bytes, 16));
        if (bytes) std::memcpy(host.data() + off, p, bytes);
        return off;
    }
    void *upload() {
        void *d = nullptr;
        hip_check(hipMalloc(&d, host.size()), "hipMalloc");
        const hipError_t err = hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice);
        if (err != hipSuccess) (void)hipFree(d);
        hip_check(err, "hipMemcpy");
        return d;
    }
};

bool finite_all(const float *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Bounding sphere of a set of spheres (AABB centre, radius = farthest reach), rounded up and
// padded by 1e-5 m so the FP32 mid-phase stays conservative.
void bounding_sphere(const std::vector<const float *> &sph, float out[4]) {
    if (sph.empty()) {
        out[0] = out[1] = out[2] = 0.0f;
        out[3] = -1.0f;
        return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (const float *s : sph)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], (double)s[a] - s[3]);
            hi[a] = std::max(hi[a], (double)s[a] + s[3]);
        }
    double c[3];
    for (int a = 0; a < 3; ++a) c[a] = 0.5 * (lo[a] + hi[a]);
    double R = 0.0;
    for (const float *s : sph) {
        const double dx = s[0] - c[0], dy = s[1] - c[1], dz = s[2] - c[2];
        R = std::max(R, std::sqrt(dx * dx + dy * dy + dz * dz) + s[3]);
    }
    for (int a = 0; a < 3; ++a) out[a] = (float)c[a];
    out[3] = std::nextafter((float)(R + 1e-5), INFINITY);
}

// Distance from point x to the segment p + s u, s in [0, 1] (double).
double point_segment(const double x[3], const double p[3], const double u[3]) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double s = 0.0;
    if (uu > 0.0) s = std::min(1.0, std::max(0.0, ((x[0] - p[0]) * u[0] + (x[1] - p[1]) * u[1] +
                                                  (x[2] - p[2]) * u[2]) / uu));
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double v = x[a] - p[a] - s * u[a];
        d2 += v * v;
    }
    return std::sqrt(d2);
}

// Bounding capsule of a set of spheres about their bounding sphere's centre c (st.coarse): the
// segment c - h .. c + h, whose axis is the principal direction of the centres (power iteration
// on their covariance) or, if that gives a smaller radius, the direction of the two farthest
// centres; |h| reaches the farthest projection of a centre.  Written to a StepRec.
void bounding_capsule(const std::vector<const float *> &sph, StepRec &st) {
    const size_t n = sph.size();
    const double c[3] = {st.coarse[0], st.coarse[1], st.coarse[2]};
    auto fit = [&](const double axis[3], double h[3]) {
        double len = 0.0;
        for (const float *s : sph)
            len = std::max(len, std::fabs((s[0] - c[0]) * axis[0] + (s[1] - c[1]) * axis[1] +
                                          (s[2] - c[2]) * axis[2]));
        double p[3], u[3];
        for (int a = 0; a < 3; ++a) {
            h[a] = len * axis[a];
            p[a] = c[a] - h[a];
            u[a] = 2.0 * h[a];
        }
        double r = 0.0;
        for (const float *s : sph) {
            const double x[3] = {s[0], s[1], s[2]};
            r = std::max(r, point_segment(x, p, u) + s[3]);
        }
        return r;
    };
    double best_h[3] = {0, 0, 0}, best_r = 1e300;
    std::vector<std::array<double, 3>> axes;
    {   // principal direction
        double m[3] = {0, 0, 0}, C[3][3] = {{0}};
        for (const float *s : sph)
            for (int a = 0; a < 3; ++a) m[a] += s[a] / (double)n;
        for (const float *s : sph)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) C[a][b] += (s[a] - m[a]) * (s[b] - m[b]);
        double v[3] = {1.0, 0.7, 0.3};
        for (int it = 0; it < 200; ++it) {
            double w[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) w[a] += C[a][b] * v[b];
            const double nw = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            if (!(nw > 0.0)) break;
            for (int a = 0; a < 3; ++a) v[a] = w[a] / nw;
        }
        const double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        axes.push_back({v[0] / nv, v[1] / nv, v[2] / nv});
    }
    {   // farthest pair of centres
        double best = 0.0, ax[3] = {1, 0, 0};
        for (size_t i = 0; i < n; ++i)
            for (size_t j = i + 1; j < n; ++j) {
                double d[3], dd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    d[a] = (double)sph[j][a] - sph[i][a];
                    dd += d[a] * d[a];
                }
                if (dd > best) {
                    best = dd;
                    for (int a = 0; a < 3; ++a) ax[a] = d[a] / std::sqrt(dd);
                }
            }
        axes.push_back({ax[0], ax[1], ax[2]});
    }
    for (const auto &ax : axes) {
        double h[3];
        const double r = fit(ax.data(), h);
        if (r < best_r) {
            best_r = r;
            for (int a = 0; a < 3; ++a) best_h[a] = h[a];
        }
    }
    double hh = 0.0;
    for (int a = 0; a < 3; ++a) {
        st.cap_h[a] = (float)best_h[a];
        hh += (double)st.cap_h[a] * st.cap_h[a];
    }
    // the float-rounded segment moves by at most a few 1e-8 m; the 1 mm padding covers it
    st.cap_r = std::nextafter((float)(best_r + 1e-3), INFINITY);
    // h rotated to the world frame and stored as three halves rounded toward zero: each
    // component is off by less than 2^-10 of |h| (plus 2^-24 for a subnormal half), so the
    // stored segment lies within sqrt(3) (2^-10 |h| + 2^-24) of the exact one
    const double herr = std::sqrt(3.0) * (std::ldexp(std::sqrt(hh), -10) + std::ldexp(1.0, -24));
    st.cap_rq = std::nextafter((float)((double)st.cap_r + herr + 1e-6), INFINITY);
    st.cap_uu = (float)(4.0 * hh);
    st.cap_inv = hh > 0.0 ? (float)(1.0 / (4.0 * hh)) : 0.0f;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Robot
// ---------------------------------------------------------------------------------------------
struct vk_robot_s {
    int device = 0;
    void *blob = nullptr;
    RobotDev dev{};
    int dof = 0, n_spheres = 0;
    // the program records on the host (the source of a specialised program)
    std::vector<StepRec> steps;
    std::vector<BlockRec> blocks;
    std::vector<EntryRec> entries;
    std::vector<JointRec> path_recs;
    std::vector<float4> spheres;
    // kernels compiled for this robot (vk_robot_specialize) and whether calls use them
    hipModule_t module = nullptr;
    SpecEdgeKernels spec{};
    std::atomic<int> use_spec{0};
    // launch settings of this robot's calls (set by the autotuner or the caller)
    std::atomic<int> edge_block{kDefaultEdgeBlock}, edge_bpc{kDefaultEdgeBpc};
    std::atomic<int> edge_tickets{kDefaultTickets};
    std::atomic<int> edge_parts{1};    // waves sharing one edge's rake (long edges)
    std::atomic<int> edge_ranges{-1};  // test ranges of a small edge batch: -1 automatic
    std::atomic<int> split_num{0}, split_den{1};
    std::atomic<int> max_ranges{-1};   // test ranges of a small state batch: -1 automatic
};

struct vk_env_s {
    int device = 0;
    void *blob = nullptr;
    EnvDev dev{};
    int64_t n_points = 0;              // spheres kept in the point grid
    int64_t n_vlist = 0, n_field = 0;  // voxel candidate entries, clearance-field cells
    size_t host_bytes = 0;             // device memory the environment takes
};

struct vk_edge_batch_s {
    int device = 0;
    void *blob = nullptr;              // BatchSet records and the set of every edge
    unsigned long long *queue = nullptr;  // the batch's own work-queue counters
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t walk = nullptr;     // the persistent launch's node (its arrays are updated)
    vk::KernelNode reset, launch;      // the two nodes' launches and argument values
    int64_t total = 0;
    int block = 0, per_cu = 0;
};

namespace {

void build_robot(const vk_robot_desc *d, vk_robot_s *r, bool upload = true) {
    if (!d) raise(VK_ERR_INVALID_ARG, "robot desc is NULL");
    const int dof = d->dof;
    if (dof < 1) raise(VK_ERR_INVALID_ARG, "dof must be >= 1");
    if (dof > kMaxDof) raise(VK_ERR_UNSUPPORTED, "dof > 64 is not supported");
    if (!d->dh) raise(VK_ERR_INVALID_ARG, "dh is NULL");
    if (!finite_all(d->dh, (size_t)dof * 5)) raise(VK_ERR_INVALID_ARG, "dh has non-finite values");
    if (d->mount && !finite_all(d->mount, (size_t)dof * 12))
        raise(VK_ERR_INVALID_ARG, "mount has non-finite values");
    const int S = d->n_spheres, P = d->n_self_pairs;
    if (S < 0 || P < 0) raise(VK_ERR_INVALID_ARG, "negative sphere or pair count");
    if (S > 0 && (!d->sphere_link || !d->sphere_xyzr)) raise(VK_ERR_INVALID_ARG, "spheres are NULL");
    if (P > 0 && !d->self_pairs) raise(VK_ERR_INVALID_ARG, "self_pairs is NULL");

    std::vector<int> par(dof + 1, -1);      // parent link of every link
    for (int j = 0; j < dof; ++j) {
        const int p = d->parent_link ? d->parent_link[j] : j;
        if (p < 0 || p > j) raise(VK_ERR_INVALID_ARG, "parent_link[j] must be in [0, j]");
        par[j + 1] = p;
    }
    std::vector<int> first(dof + 2, 0), count(dof + 1, 0);
    for (int s = 0; s < S; ++s) {
        const int l = d->sphere_link[s];
        if (l < 0 || l > dof) raise(VK_ERR_INVALID_ARG, "sphere_link out of range");
        if (s > 0 && l < d->sphere_link[s - 1]) raise(VK_ERR_INVALID_ARG, "sphere_link must be non-decreasing");
        const float *x = d->sphere_xyzr + 4 * s;
        if (!finite_all(x, 4) || !(x[3] > 0.0f)) raise(VK_ERR_INVALID_ARG, "sphere radius must be finite and > 0");
        count[l]++;
    }
    for (int l = 0; l <= dof; ++l) first[l + 1] = first[l] + count[l];

    auto anc = [&](int link) {               // joints from the base to `link`, base-most first
        std::vector<int> v;
        while (link > 0) {
            v.push_back(link - 1);
            link = par[link];
        }
        std::reverse(v.begin(), v.end());
        return v;
    };

    std::vector<JointRec> joints(dof);
    for (int j = 0; j < dof; ++j) {
        JointRec &J = joints[j];
        std::memset(&J, 0, sizeof J);
        J.index = j;
        const float *h = d->dh + 5 * j;
        J.a = h[0];
        J.d = h[1];
        J.ca = h[2];
        J.sa = h[3];
        J.theta_off = h[4];
        J.s_off = (float)std::sin((double)h[4]);
        J.c_off = (float)std::cos((double)h[4]);
        J.prismatic = d->joint_type ? d->joint_type[j] : 0;
        if (J.prismatic != 0 && J.prismatic != 1)
            raise(VK_ERR_INVALID_ARG, "joint_type must be 0 (revolute) or 1 (prismatic)");
        J.twist = (h[2] == 1.0f && h[3] == 0.0f)    ? kTwist0
                  : (h[2] == 0.0f && h[3] == 1.0f)  ? kTwistP90
                  : (h[2] == 0.0f && h[3] == -1.0f) ? kTwistM90
                                                    : kTwistGeneral;
        J.parent = par[j + 1];
        static const float ident[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
        const float *m = d->mount ? d->mount + 12 * j : ident;
        std::memcpy(J.m, m, sizeof J.m);
        J.has_mount = std::memcmp(m, ident, sizeof ident) != 0;
    }

    // link steps in topological (index) order, spheres in chunks of at most kSpl
    std::vector<StepRec> steps;
    std::vector<int> paths;
    std::vector<int> sphere_step(S, 0), sphere_k(S, 0);
    int cur = 0;
    for (int l = 0; l <= dof; ++l) {
        const int nchunk = std::max(1, (count[l] + kSpl - 1) / kSpl);
        for (int c = 0; c < nchunk; ++c) {
            StepRec st;
            std::memset(&st, 0, sizeof st);
            st.link = l;
            st.joint = -1;
            st.restart_len = -1;
            if (c == 0 && l > 0) {
                st.joint = l - 1;
                if (par[l] != cur) {
                    std::vector<int> a = anc(par[l]);
                    st.restart_off = (int)paths.size();
                    st.restart_len = (int)a.size();
                    paths.insert(paths.end(), a.begin(), a.end());
                }
                cur = l;
            }
            st.sph_first = first[l] + c * kSpl;
            st.sph_count = std::min(kSpl, count[l] - c * kSpl);
            if (st.sph_count < 0) st.sph_count = 0;
            std::vector<const float *> sp;
            for (int k = 0; k < st.sph_count; ++k) {
                sp.push_back(d->sphere_xyzr + 4 * (st.sph_first + k));
                sphere_step[st.sph_first + k] = (int)steps.size();
                sphere_k[st.sph_first + k] = k;
            }
            bounding_sphere(sp, st.coarse);
            if (!sp.empty()) bounding_capsule(sp, st);
            steps.push_back(st);
        }
        if (l == 0 && count[0] == 0) steps.pop_back();   // nothing to do on an empty base
    }

    // self pairs: grouped by the step holding the later-link sphere, then by the step holding
    // the earlier sphere (blocks ordered by that step, so consecutive blocks tend to walk down
    // one branch and can continue from the previous block's pose)
    std::vector<std::map<int, std::map<int, uint32_t>>> grp(steps.size());
    for (int p = 0; p < P; ++p) {
        int s = d->self_pairs[2 * p], t = d->self_pairs[2 * p + 1];
        if (s < 0 || s >= S || t < 0 || t >= S) raise(VK_ERR_INVALID_ARG, "self pair index out of range");
        int ls = d->sphere_link[s], lt = d->sphere_link[t];
        if (ls == lt) raise(VK_ERR_INVALID_ARG, "self pair on a single link (rigid, not supported)");
        if (ls < lt) {
            std::swap(s, t);
            std::swap(ls, lt);
        }
        grp[sphere_step[s]][sphere_step[t]][t] |= 1u << sphere_k[s];
    }
    std::vector<BlockRec> blocks;
    std::vector<EntryRec> entries;
    for (size_t si = 0; si < steps.size(); ++si) {
        steps[si].blk_first = (int)blocks.size();
        for (auto &kv : grp[si]) {
            const int sa = kv.first;
            const int A = steps[sa].link;
            BlockRec B;
            std::memset(&B, 0, sizeof B);
            B.step_a = sa;
            B.link = A;
            steps[sa].slot = 1;           // read by a later block: numbered below
            const std::vector<int> path = anc(A);
            B.path_off = (int)paths.size();
            B.path_len = (int)path.size();
            paths.insert(paths.end(), path.begin(), path.end());
            uint64_t mask = 0;
            for (int l = par[A]; l > 0; l = par[l]) mask |= 1ull << (l - 1);
            B.anc_lo = (uint32_t)mask;
            B.anc_hi = (uint32_t)(mask >> 32);
            B.ent_first = (int)entries.size();
            std::vector<const float *> sp;
            for (auto &tm : kv.second) {
                EntryRec E;
                std::memset(&E, 0, sizeof E);
                const float *x = d->sphere_xyzr + 4 * tm.first;
                E.x = x[0];
                E.y = x[1];
                E.z = x[2];
                E.r = x[3];
                E.mask = tm.second;
                // entry gate against this step's bound, and the pair constants (see the self
                // test of the walk): r r_k for paired spheres, -inf for the others
                const double g = (double)x[3] + (double)steps[si].coarse[3];
                E.gate2 = std::nextafter((float)(g * g), INFINITY);
                E.nhr2 = (float)(-0.5 * (double)x[3] * (double)x[3]);
                for (int k = 0; k < kSpl; ++k)
                    E.rr[k] = (k < steps[si].sph_count && ((tm.second >> k) & 1u))
                                  ? x[3] * d->sphere_xyzr[4 * (steps[si].sph_first + k) + 3]
                                  : -INFINITY;
                entries.push_back(E);
                sp.push_back(x);
            }
            B.ent_count = (int)kv.second.size();
            blocks.push_back(B);
        }
        steps[si].blk_count = (int)blocks.size() - steps[si].blk_first;
    }
    // walk-cache slots: only the steps a later block reads keep their bounds per lane
    int n_slots = 0;
    for (StepRec &st : steps) st.slot = st.slot ? n_slots++ : -1;
    for (StepRec &st : steps)
        if (st.joint >= 0) st.jr = joints[st.joint];
    for (BlockRec &B : blocks) {
        const StepRec &A = steps[B.step_a];
        B.slot_a = A.slot;
        B.ra = A.coarse[3];
        B.rqa = A.cap_rq;
    }

    std::vector<float4> spheres(S + kSpl, make_float4(0, 0, 0, 0));   // kSpl padding records
    for (int s = 0; s < S; ++s)
        spheres[s] = make_float4(d->sphere_xyzr[4 * s], d->sphere_xyzr[4 * s + 1],
                                 d->sphere_xyzr[4 * s + 2], d->sphere_xyzr[4 * s + 3]);
    if (paths.empty()) paths.push_back(0);

    std::vector<JointRec> path_recs(paths.size());
    for (size_t i = 0; i < paths.size(); ++i) path_recs[i] = joints[std::min<int>(paths[i], dof - 1)];
    r->steps = steps;
    r->blocks = blocks;
    r->entries = entries;
    r->path_recs = path_recs;
    r->spheres = spheres;
    r->dof = dof;
    r->n_spheres = S;
    r->dev.dof = dof;
    r->dev.n_steps = (int)steps.size();
    r->dev.n_slots = n_slots;
    r->dev.n_tests = (int)(steps.size() + blocks.size());
    r->dev.n_spheres = S;
    r->dev.n_links = dof + 1;
    if (!upload) return;

    Blob b;
    const size_t o_j = b.add(joints.data(), joints.size() * sizeof(JointRec));
    const size_t o_s = b.add(steps.data(), steps.size() * sizeof(StepRec));
    const size_t o_b = b.add(blocks.data(), blocks.size() * sizeof(BlockRec));
    const size_t o_e = b.add(entries.data(), entries.size() * sizeof(EntryRec));
    const size_t o_p = b.add(paths.data(), paths.size() * sizeof(int));
    const size_t o_pr = b.add(path_recs.data(), path_recs.size() * sizeof(JointRec));
    const size_t o_sp = b.add(spheres.data(), spheres.size() * sizeof(float4));
    const size_t o_ss = b.add(sphere_step.data(), sphere_step.size() * sizeof(int));
    r->device = current_device();
    r->blob = b.upload();
    char *base = static_cast<char *>(r->blob);
    r->dev.joints = reinterpret_cast<const JointRec *>(base + o_j);
    r->dev.steps = reinterpret_cast<const StepRec *>(base + o_s);
    r->dev.blocks = reinterpret_cast<const BlockRec *>(base + o_b);
    r->dev.entries = reinterpret_cast<const EntryRec *>(base + o_e);
    r->dev.paths = reinterpret_cast<const int32_t *>(base + o_p);
    r->dev.path_recs = reinterpret_cast<const JointRec *>(base + o_pr);
    r->dev.spheres = reinterpret_cast<const float4 *>(base + o_sp);
    r->dev.sphere_step = reinterpret_cast<const int32_t *>(base + o_ss);
}

float int_bits(int v) {
    float f;
    std::memcpy(&f, &v, sizeof f);
    return f;
}

constexpr int kGridMinSpheres = 1024;
constexpr double kGridRobotR = 0.08;   // robot radius the point-grid cell size is tuned for
constexpr double kFieldCell = 0.015;   // clearance-field cell edge (m)
constexpr double kFieldStep = 0.0005;  // clearance-field unit (m): it reaches 255 x 0.5 mm
constexpr int64_t kFieldMaxCells = int64_t(1) << 23;
constexpr double kUnitTol = 1e-5;      // unit axes and orthonormal rotations, within this
constexpr double kVoxCap = 0.5;        // voxel lists cover link bounding spheres up to 0.5 m
constexpr double kVoxMinCell = 0.05;
constexpr double kVoxMaxCells = 49152; // byte field of at most 48 KiB (fits LDS with records)

// Host-side signed distances (double) used only to build the voxel lists.
struct HostPrim {
    int type, idx;
    double v[15];
    double bc[3], br;              // bounding sphere
};

double host_sd(const HostPrim &p, const double *x) {
    const double *v = p.v;
    auto nrm = [](double a, double b, double c) { return std::sqrt(a * a + b * b + c * c); };
    switch (p.type) {
    case 0:
        return nrm(x[0] - v[0], x[1] - v[1], x[2] - v[2]) - v[3];
    case 1: {
        const double u[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        const double w[3] = {x[0] - v[0], x[1] - v[1], x[2] - v[2]};
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double t = uu > 0.0 ? (w[0] * u[0] + w[1] * u[1] + w[2] * u[2]) / uu : 0.0;
        t = std::min(1.0, std::max(0.0, t));
        return nrm(w[0] - t * u[0], w[1] - t * u[1], w[2] - t * u[2]) - v[6];
    }
    case 2: {
        const double r[3] = {x[0] - v[0], x[1] - v[1], x[2] - v[2]};
        const double h = r[0] * v[3] + r[1] * v[4] + r[2] * v[5];
        const double rho = nrm(r[0] - h * v[3], r[1] - h * v[4], r[2] - h * v[5]);
        const double a = std::fabs(h) - v[6], b = rho - v[7];
        if (a <= 0.0 && b <= 0.0) return std::max(a, b);
        return nrm(std::max(a, 0.0), std::max(b, 0.0), 0.0);
    }
    default: {
        const double r[3] = {x[0] - v[0], x[1] - v[1], x[2] - v[2]};
        double q[3], o = 0.0, m = -1e300;
        for (int k = 0; k < 3; ++k) {
            const double pk = v[3 + k] * r[0] + v[6 + k] * r[1] + v[9 + k] * r[2];
            q[k] = std::fabs(pk) - v[12 + k];
            o += std::max(q[k], 0.0) * std::max(q[k], 0.0);
            m = std::max(m, q[k]);
        }
        return std::sqrt(o) + std::min(m, 0.0);
    }
    }
}

void build_env(const vk_env_desc *d, vk_env_s *e, bool upload = true) {
    if (!d) raise(VK_ERR_INVALID_ARG, "env desc is NULL");
    const int ns = d->n_spheres, nc = d->n_capsules, ny = d->n_cylinders, nb = d->n_boxes;
    if (ns < 0 || nc < 0 || ny < 0 || nb < 0) raise(VK_ERR_INVALID_ARG, "negative primitive count");
    if ((ns && !d->spheres) || (nc && !d->capsules) || (ny && !d->cylinders) || (nb && !d->boxes))
        raise(VK_ERR_INVALID_ARG, "primitive array is NULL");
    if ((ns && !finite_all(d->spheres, (size_t)ns * 4)) ||
        (nc && !finite_all(d->capsules, (size_t)nc * 7)) ||
        (ny && !finite_all(d->cylinders, (size_t)ny * 8)) ||
        (nb && !finite_all(d->boxes, (size_t)nb * 15)))
        raise(VK_ERR_INVALID_ARG, "primitive values must be finite");
    for (int i = 0; i < ns; ++i)
        if (d->spheres[4 * i + 3] < 0.0f) raise(VK_ERR_INVALID_ARG, "negative sphere radius");
    // the voxel bounds and the link-sphere gate need a 1-Lipschitz signed distance: a unit
    // cylinder axis and an orthonormal box rotation (within FP32 rounding of the input)
    for (int i = 0; i < ny; ++i) {
        const float *w = d->cylinders + 8 * i + 3;
        const double len = std::sqrt((double)w[0] * w[0] + (double)w[1] * w[1] + (double)w[2] * w[2]);
        if (std::fabs(len - 1.0) > kUnitTol) raise(VK_ERR_INVALID_ARG, "cylinder axis is not a unit vector");
    }
    for (int i = 0; i < nb; ++i) {
        const float *R = d->boxes + 15 * i + 3;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double g = 0.0;               // (R^T R)[a][b]: columns a and b of R
                for (int k = 0; k < 3; ++k) g += (double)R[3 * k + a] * R[3 * k + b];
                if (std::fabs(g - (a == b ? 1.0 : 0.0)) > kUnitTol)
                    raise(VK_ERR_INVALID_ARG, "box rotation is not orthonormal");
            }
    }

    // Large sets of small spheres (point clouds) go to a uniform grid: when there are more than
    // kGridMinSpheres spheres, those with a radius at most twice the median radius.
    std::vector<char> in_grid(ns, 0);
    std::vector<int> grid_idx;
    float gmax_r = 0.0f;
    if (ns > kGridMinSpheres) {
        std::vector<float> radii(ns);
        for (int i = 0; i < ns; ++i) radii[i] = d->spheres[4 * i + 3];
        std::nth_element(radii.begin(), radii.begin() + ns / 2, radii.end());
        const float lim = 2.0f * radii[ns / 2];
        for (int i = 0; i < ns; ++i)
            if (d->spheres[4 * i + 3] <= lim) {
                in_grid[i] = 1;
                grid_idx.push_back(i);
                gmax_r = std::max(gmax_r, d->spheres[4 * i + 3]);
            }
    }

    // primitive records (the voxel lists refer to them by type and index)
    std::vector<float4> sph, cap, cyl, box;
    std::vector<HostPrim> prims;
    for (int i = 0; i < ns; ++i) {
        if (in_grid[i]) continue;
        const float *q = d->spheres + 4 * i;
        HostPrim p{0, (int)sph.size(), {}, {q[0], q[1], q[2]}, q[3]};
        for (int k = 0; k < 4; ++k) p.v[k] = q[k];
        prims.push_back(p);
        sph.push_back(make_float4(q[0], q[1], q[2], q[3]));
    }
    for (int i = 0; i < nc; ++i) {
        const float *q = d->capsules + 7 * i;
        HostPrim p{1, i, {}, {}, 0.0};
        for (int k = 0; k < 7; ++k) p.v[k] = q[k];
        double hl = 0.0;
        for (int a = 0; a < 3; ++a) {
            p.bc[a] = 0.5 * ((double)q[a] + q[3 + a]);
            hl += 0.25 * ((double)q[3 + a] - q[a]) * ((double)q[3 + a] - q[a]);
        }
        p.br = std::sqrt(hl) + q[6];
        prims.push_back(p);
        const float ux = q[3] - q[0], uy = q[4] - q[1], uz = q[5] - q[2];
        const float uu = ux * ux + uy * uy + uz * uz;
        cap.push_back(make_float4(q[0], q[1], q[2], q[6]));
        cap.push_back(make_float4(ux, uy, uz, uu > 0.0f ? 1.0f / uu : 0.0f));
    }
    for (int i = 0; i < ny; ++i) {
        const float *q = d->cylinders + 8 * i;
        HostPrim p{2, i, {}, {q[0], q[1], q[2]}, std::hypot((double)q[6], (double)q[7])};
        for (int k = 0; k < 8; ++k) p.v[k] = q[k];
        prims.push_back(p);
        cyl.push_back(make_float4(q[0], q[1], q[2], q[6]));
        cyl.push_back(make_float4(q[3], q[4], q[5], q[7]));
    }
    for (int i = 0; i < nb; ++i) {
        const float *b = d->boxes + 15 * i;
        HostPrim p{3, i, {}, {b[0], b[1], b[2]},
                   std::sqrt((double)b[12] * b[12] + (double)b[13] * b[13] + (double)b[14] * b[14])};
        for (int k = 0; k < 15; ++k) p.v[k] = b[k];
        prims.push_back(p);
        const float *R = b + 3, *ext = b + 12;
        for (int k = 0; k < 3; ++k) box.push_back(make_float4(R[k], R[3 + k], R[6 + k], ext[k]));
        box.push_back(make_float4(b[0], b[1], b[2], 0.0f));
    }

    // voxel broadphase: grid over everything within kVoxCap of a primitive
    std::memset(&e->dev, 0, sizeof e->dev);
    std::vector<int> vstart(1, 0);
    std::vector<int2> vlist;
    std::vector<unsigned char> vdist;
    if (!prims.empty()) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (const HostPrim &p : prims)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], p.bc[a] - p.br - kVoxCap);
                hi[a] = std::max(hi[a], p.bc[a] + p.br + kVoxCap);
            }
        const double vol = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        const double h = std::max(kVoxMinCell, std::cbrt(vol / kVoxMaxCells) * 1.0001);
        int dim[3];
        for (int a = 0; a < 3; ++a) dim[a] = std::max(1, (int)std::ceil((hi[a] - lo[a]) / h));
        const int64_t nvox = (int64_t)dim[0] * dim[1] * dim[2];
        const double hd = 0.5 * h * std::sqrt(3.0);
        std::vector<std::vector<std::pair<float, int>>> cells(nvox);
        for (size_t pi = 0; pi < prims.size(); ++pi) {
            const HostPrim &p = prims[pi];
            int c0[3], c1[3];
            for (int a = 0; a < 3; ++a) {
                c0[a] = std::max(0, (int)std::floor((p.bc[a] - p.br - kVoxCap - hd - lo[a]) / h));
                c1[a] = std::min(dim[a] - 1, (int)std::floor((p.bc[a] + p.br + kVoxCap + hd - lo[a]) / h));
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) {
                        const double ctr[3] = {lo[0] + (x + 0.5) * h, lo[1] + (y + 0.5) * h,
                                               lo[2] + (z + 0.5) * h};
                        // every point of the cell is within hd of its centre (1-Lipschitz sd)
                        const double lb = host_sd(p, ctr) - hd - 1e-5;
                        if (lb < kVoxCap)
                            cells[((int64_t)z * dim[1] + y) * dim[0] + x].push_back(
                                {(float)std::nextafter((float)lb, -INFINITY),
                                 (p.type << 28) | p.idx});
                    }
        }
        const double q = kVoxCap / 255.0;
        vdist.resize((size_t)nvox);
        for (int64_t c = 0; c < nvox; ++c) {
            auto &L = cells[c];
            std::sort(L.begin(), L.end());
            for (auto &it : L) vlist.push_back(make_int2(it.second, 0));
            for (size_t k = 0; k < L.size(); ++k) {
                float f = L[k].first;
                std::memcpy(&vlist[vlist.size() - L.size() + k].y, &f, sizeof f);
            }
            vstart.push_back((int)vlist.size());
            const double m = L.empty() ? kVoxCap : std::max(0.0, (double)L[0].first);
            vdist[c] = (unsigned char)std::min(255.0, std::floor(m / q));
        }
        if (vlist.size() >= (size_t(1) << 31)) raise(VK_ERR_UNSUPPORTED, "voxel lists too large");
        for (int a = 0; a < 3; ++a) {
            e->dev.vdim[a] = dim[a];
            e->dev.vorg[a] = (float)lo[a];
        }
        e->dev.n_vox = (int)nvox;
        e->dev.vinv = (float)(1.0 / h);
        e->dev.vq = (float)q;
        e->dev.vcap = (float)kVoxCap;
    }

    std::vector<float4> rec;
    auto put = [&](const std::vector<float4> &v) {
        const int off = (int)rec.size();
        rec.insert(rec.end(), v.begin(), v.end());
        return off;
    };
    e->dev.off_sph = put(sph);
    e->dev.off_cap = put(cap);
    e->dev.off_cyl = put(cyl);
    e->dev.off_box = put(box);

    // point grid: cell size sized so robot spheres up to kGridRobotR scan a 3x3x3 neighbourhood
    std::vector<float4> pts;
    std::vector<uint8_t> pfield;
    GridDev gd;
    std::memset(&gd, 0, sizeof gd);
    if (!grid_idx.empty()) {
        const double h = kGridRobotR + gmax_r;
        double glo[3] = {1e300, 1e300, 1e300}, ghi[3] = {-1e300, -1e300, -1e300};
        for (int i : grid_idx)
            for (int a = 0; a < 3; ++a) {
                glo[a] = std::min(glo[a], (double)d->spheres[4 * i + a]);
                ghi[a] = std::max(ghi[a], (double)d->spheres[4 * i + a]);
            }
        int dim[3];
        for (int a = 0; a < 3; ++a) {
            glo[a] -= 1e-3;
            dim[a] = (int)std::floor((ghi[a] - glo[a]) / h) + 1;
        }
        const int64_t ncell = (int64_t)dim[0] * dim[1] * dim[2];
        if (ncell > (int64_t(1) << 24)) raise(VK_ERR_UNSUPPORTED, "point cloud grid too large");
        auto cell_of = [&](int i) {
            int c[3];
            for (int a = 0; a < 3; ++a) {
                int v = (int)std::floor(((double)d->spheres[4 * i + a] - glo[a]) / h);
                c[a] = std::min(std::max(v, 0), dim[a] - 1);
            }
            return ((int64_t)c[2] * dim[1] + c[1]) * dim[0] + c[0];
        };
        std::vector<int> start(ncell + 1, 0);
        for (int i : grid_idx) start[cell_of(i) + 1]++;
        for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
        std::vector<int> fill(start.begin(), start.end() - 1);
        pts.resize(grid_idx.size());
        for (int i : grid_idx) {
            const float *q = d->spheres + 4 * i;
            pts[fill[cell_of(i)]++] = make_float4(q[0], q[1], q[2], q[3]);
        }
        std::vector<float4> cells((ncell + 1 + 3) / 4, make_float4(0, 0, 0, 0));
        std::memcpy(cells.data(), start.data(), start.size() * sizeof(int));
        e->dev.off_cell = put(cells);
        e->dev.n_cells = (int)ncell;
        gd.n_pts = (int)pts.size();
        e->n_points = (int64_t)pts.size();
        for (int a = 0; a < 3; ++a) {
            gd.gdim[a] = dim[a];
            gd.gorg[a] = (float)glo[a];
        }
        gd.ginv = (float)(1.0 / h);
        gd.gmax_r = gmax_r;

        // clearance field: 1.5 cm cells (coarser for a very large cloud) over the points' box
        // widened by their largest radius plus the field's reach, so that a location outside it
        // is farther than the reach from every point
        const double reach = 255.0 * kFieldStep;
        double plo[3], phi[3], cell = kFieldCell;
        for (int a = 0; a < 3; ++a) {
            plo[a] = glo[a] + 1e-3 - gmax_r - reach;
            phi[a] = ghi[a] + gmax_r + reach;
        }
        int pd[3];
        for (;;) {
            for (int a = 0; a < 3; ++a) pd[a] = (int)std::ceil((phi[a] - plo[a]) / cell);
            if ((int64_t)pd[0] * pd[1] * pd[2] <= kFieldMaxCells) break;
            cell *= 1.25;
        }
        std::vector<float> clear((size_t)pd[0] * pd[1] * pd[2], (float)reach);
        for (int i : grid_idx) {
            const double p[3] = {d->spheres[4 * i], d->spheres[4 * i + 1], d->spheres[4 * i + 2]};
            const double rp = d->spheres[4 * i + 3];
            int c0[3], c1[3];
            for (int a = 0; a < 3; ++a) {
                c0[a] = std::max(0, (int)std::floor((p[a] - rp - reach - plo[a]) / cell));
                c1[a] = std::min(pd[a] - 1, (int)std::floor((p[a] + rp + reach - plo[a]) / cell));
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) {
                        const int c[3] = {x, y, z};
                        double d2 = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            const double g = plo[a] + (c[a] + 0.5) * cell - p[a];
                            d2 += g * g;
                        }
                        float &v = clear[((size_t)z * pd[1] + y) * pd[0] + x];
                        v = std::min(v, (float)(std::sqrt(d2) - rp));
                    }
        }
        // rounded down, less 10 um for the device's FP32 distance to the cell centre
        pfield.resize(clear.size());
        for (size_t c = 0; c < clear.size(); ++c) {
            const double u = std::floor(((double)clear[c] - 1e-5) / kFieldStep);
            pfield[c] = (uint8_t)std::min(255.0, std::max(0.0, u));
        }
        for (int a = 0; a < 3; ++a) {
            gd.pdim[a] = pd[a];
            gd.porg[a] = (float)plo[a];
        }
        gd.pinv = (float)(1.0 / cell);
        gd.pcell = (float)cell;
        gd.pq = std::nextafter((float)kFieldStep, 0.0f);
    } else {
        e->dev.off_cell = (int)rec.size();
    }
    // the voxel byte field goes last: it is read from global memory (one byte per lane and
    // link), so it never competes for LDS with the primitives and the cell index
    {
        std::vector<float4> packed((vdist.size() + 15) / 16, make_float4(0, 0, 0, 0));
        if (!vdist.empty()) std::memcpy(packed.data(), vdist.data(), vdist.size());
        e->dev.off_vdist = put(packed);
    }
    e->dev.n_rec = (int)rec.size();
    e->dev.n_sph = (int)sph.size();
    e->dev.n_cap = nc;
    e->dev.n_cyl = ny;
    e->dev.n_box = nb;
    if (rec.empty()) rec.push_back(make_float4(0, 0, 0, 0));
    Blob bl;
    const size_t o_r = bl.add(rec.data(), rec.size() * sizeof(float4));
    const size_t o_p = bl.add(pts.data(), pts.size() * sizeof(float4));
    const size_t o_s = bl.add(vstart.data(), vstart.size() * sizeof(int));
    const size_t o_l = bl.add(vlist.data(), vlist.size() * sizeof(int2));
    const size_t o_f = bl.add(pfield.data(), pfield.size());
    const size_t o_g = bl.add(&gd, sizeof gd);     // its pointers are set after the upload
    e->host_bytes = bl.host.size();
    e->n_vlist = (int64_t)vlist.size();
    e->n_field = (int64_t)pfield.size();
    if (!upload) return;
    e->device = current_device();
    e->blob = bl.upload();
    char *base = static_cast<char *>(e->blob);
    e->dev.rec = reinterpret_cast<const float4 *>(base + o_r);
    if (e->dev.n_cells > 0) {
        gd.pts = reinterpret_cast<const float4 *>(base + o_p);
        gd.pfield = reinterpret_cast<const uint8_t *>(base + o_f);
        hip_check(hipMemcpy(base + o_g, &gd, sizeof gd, hipMemcpyHostToDevice), "hipMemcpy");
        e->dev.grid = reinterpret_cast<const GridDev *>(base + o_g);
    }
    e->dev.vstart = reinterpret_cast<const int32_t *>(base + o_s);
    e->dev.vlist = reinterpret_cast<const int2 *>(base + o_l);
}

// Environment for one launch, with the number of leading records staged in LDS: the
// primitives and the point-grid cell index when both fit, else the primitives alone, else none
// (everything read from global memory).  `extra` is the kernel's other dynamic LDS (step
// caches, adjoint slots) and must fit on its own.
EnvDev env_for_launch(const vk_env_s *e, size_t extra) {
    const DeviceInfo &di = device_info(e->device);
    if (extra > di.max_lds) raise(VK_ERR_UNSUPPORTED, "robot too large for the LDS walk cache");
    EnvDev d = e->dev;
    auto fits = [&](int n) {
        const size_t b = (size_t)n * 16;
        return n > 0 && b <= 64 * 1024 && b + extra <= di.max_lds;
    };
    d.n_stage = fits(d.off_vdist) ? d.off_vdist : fits(d.off_cell) ? d.off_cell : 0;
    return d;
}

void check_launch(int block_threads, int blocks_per_cu, int tickets_per_wave) {
    if (block_threads < 64 || block_threads > 1024 || block_threads % 64)
        raise(VK_ERR_INVALID_ARG, "block_threads must be a multiple of 64 in [64, 1024]");
    if (blocks_per_cu < 1 || blocks_per_cu > 64)
        raise(VK_ERR_INVALID_ARG, "blocks_per_cu must be in [1, 64]");
    if (tickets_per_wave < 1 || tickets_per_wave > 64)
        raise(VK_ERR_INVALID_ARG, "tickets_per_wave must be in [1, 64]");
}

void check_pair(vk_robot r, vk_env e) {
    if (!r) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
    if (!e) raise(VK_ERR_INVALID_ARG, "env handle is NULL");
}

void check_batch(int64_t n, int64_t ld, const void *in, const void *out, const char *what) {
    if (n < 0) raise(VK_ERR_INVALID_ARG, std::string(what) + ": n < 0");
    if (n > 0 && (!in || !out)) raise(VK_ERR_INVALID_ARG, std::string(what) + ": NULL array");
    if (ld < n) raise(VK_ERR_SHAPE, std::string(what) + ": leading dimension < n");
    if (n >= (int64_t(1) << 40)) raise(VK_ERR_SHAPE, std::string(what) + ": n too large");
}


// ---- autotuner helpers ------------------------------------------------------------------------
// Median launch time (ms) of `launch` on stream s: one untimed run, then 7 runs each bracketed
// by events.
template <class F>
double time_median(hipStream_t s, F &&launch) {
    launch();
    hip_check(hipStreamSynchronize(s), "autotune sync");
    constexpr int kReps = 7;
    hipEvent_t ev[kReps + 1];
    int made = 0;
    std::vector<float> ms;
    try {
        for (; made < kReps + 1; ++made) hip_check(hipEventCreate(&ev[made]), "hipEventCreate");
        hip_check(hipEventRecord(ev[0], s), "hipEventRecord");
        for (int r = 0; r < kReps; ++r) {
            launch();
            hip_check(hipEventRecord(ev[r + 1], s), "hipEventRecord");
        }
        hip_check(hipEventSynchronize(ev[kReps]), "hipEventSynchronize");
        for (int r = 0; r < kReps; ++r) {
            float t = 0.0f;
            hip_check(hipEventElapsedTime(&t, ev[r], ev[r + 1]), "hipEventElapsedTime");
            ms.push_back(t);
        }
    } catch (...) {
        for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
        throw;
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    std::sort(ms.begin(), ms.end());
    return ms[kReps / 2];
}

int64_t pow2_bucket(int64_t x) {
    int64_t b = 1;
    while (b < x) b *= 2;
    return b;
}

// Workload class of a tuning result: the device, the robot's size, the environment's size and
// the batch size (powers of two), so that a later process reuses it without timing.
std::string tune_key(const char *what, vk_robot r, vk_env e, int64_t n) {
    hipDeviceProp_t prop{};
    hip_check(hipGetDeviceProperties(&prop, r->device), "hipGetDeviceProperties");
    std::string arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ' || c == '"' || c == '|') c = '_';
    const EnvDev &d = e->dev;
    const int64_t prims = (int64_t)d.n_sph + d.n_cap + d.n_cyl + d.n_box + (d.grid ? e->n_points : 0);
    return std::string(what) + "|" + arch + "|cu" + std::to_string(prop.multiProcessorCount) +
           "|dof" + std::to_string(r->dof) + "|s" + std::to_string(pow2_bucket(r->n_spheres)) +
           "|p" + std::to_string(pow2_bucket(std::max<int64_t>(prims, 1))) + "|n" +
           std::to_string(pow2_bucket(n));
}

// The cache file is a JSON object of objects of numbers, e.g.
//   {"edges|gfx950|cu256|dof7|s64|p256|n65536": {"block": 1024, "per_cu": 2, "tickets": 8, "ms": 0.61}}
// A file that does not parse as that is treated as empty (its workloads are timed again and it
// is rewritten).
using TuneEntry = std::map<std::string, double>;
using TuneCache = std::map<std::string, TuneEntry>;

struct JsonIn {
    const std::string &t;
    size_t i = 0;
    void ws() {
        while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < t.size() && t[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string &out) {
        if (!eat('"')) return false;
        out.clear();
        while (i < t.size() && t[i] != '"') {
            if (t[i] == '\\') return false;     // keys written here have no escapes
            out += t[i++];
        }
        return eat('"');
    }
    bool num(double &x) {
        ws();
        char *end = nullptr;
        x = std::strtod(t.c_str() + i, &end);
        if (end == t.c_str() + i) return false;
        i = (size_t)(end - t.c_str());
        return true;
    }
};

TuneCache load_tune_cache(const char *path) {
    TuneCache c;
    if (!path || !*path) return c;
    FILE *f = std::fopen(path, "rb");
    if (!f) return c;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    JsonIn in{text};
    TuneCache out;
    if (!in.eat('{')) return c;
    if (in.eat('}')) return out;
    do {
        std::string key;
        if (!in.str(key) || !in.eat(':') || !in.eat('{')) return c;
        TuneEntry e;
        if (!in.eat('}')) {
            do {
                std::string name;
                double x;
                if (!in.str(name) || !in.eat(':') || !in.num(x)) return c;
                e[name] = x;
            } while (in.eat(','));
            if (!in.eat('}')) return c;
        }
        out[key] = e;
    } while (in.eat(','));
    if (!in.eat('}')) return c;
    return out;
}

void save_tune_cache(const char *path, const TuneCache &c) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) raise(VK_ERR_INVALID_ARG, std::string("cannot write the autotune cache ") + path);
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : c) {
        std::fprintf(f, " \"%s\": {", kv.first.c_str());
        size_t j = 0;
        for (const auto &fv : kv.second)
            std::fprintf(f, "%s\"%s\": %.9g", j++ ? ", " : "", fv.first.c_str(), fv.second);
        std::fprintf(f, "}%s\n", ++i < c.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0)
        raise(VK_ERR_INVALID_ARG, std::string("cannot write the autotune cache ") + path);
}

// Field `name` of a cache entry as an int, or -1 when it is missing or not an integer.
int entry_int(const TuneEntry &e, const char *name) {
    auto it = e.find(name);
    if (it == e.end() || !(it->second == std::floor(it->second)) || std::fabs(it->second) > 1e6)
        return -1;
    return (int)it->second;
}


// ---- per-robot specialisation ----------------------------------------------------------------
// The robot's program records written out as constant arrays of a struct R (exact: floats as
// hexadecimal literals), and the persistent edge kernels instantiated on SpecProg<R>.  The
// runtime compiler builds this source with the walk's headers, embedded in the library.
std::string lit(float x) {
    if (std::isnan(x)) return "__builtin_nanf(\"\")";
    if (std::isinf(x)) return x > 0 ? "__builtin_inff()" : "-__builtin_inff()";
    char b[48];
    std::snprintf(b, sizeof b, "%af", (double)x);
    return b;
}

template <class T>
std::string lits(const T *x, int n) {
    std::string o = "{";
    for (int i = 0; i < n; ++i) o += (i ? ", " : "") + lit(x[i]);
    return o + "}";
}

std::string joint_lit(const JointRec &J) {
    static_assert(sizeof(JointRec) == 96, "JointRec fields changed: update joint_lit");
    return "{" + lit(J.a) + ", " + lit(J.d) + ", " + lit(J.ca) + ", " + lit(J.sa) + ", " +
           lit(J.theta_off) + ", " + lit(J.s_off) + ", " + lit(J.c_off) + ", " +
           std::to_string(J.twist) + ", " + std::to_string(J.has_mount) + ", " +
           std::to_string(J.parent) + ", " + std::to_string(J.prismatic) + ", " + lits(J.m, 12) +
           ", " + std::to_string(J.index) + "}";
}

std::string step_lit(const StepRec &S) {
    static_assert(sizeof(StepRec) == 192, "StepRec fields changed: update step_lit");
    const int iv[8] = {S.joint, S.restart_off, S.restart_len, S.sph_first, S.sph_count,
                       S.blk_first, S.blk_count, S.link};
    std::string o = "{";
    for (int v : iv) o += std::to_string(v) + ", ";
    return o + lits(S.coarse, 4) + ", " + lits(S.cap_h, 3) + ", " + lit(S.cap_r) + ", " +
           lit(S.cap_rq) + ", " + lit(S.cap_uu) + ", " + lit(S.cap_inv) + ", " +
           std::to_string(S.slot) + ", " + lits(S.pad, 4) + ", " + joint_lit(S.jr) + "}";
}

std::string block_lit(const BlockRec &B) {
    static_assert(sizeof(BlockRec) == 48, "BlockRec fields changed: update block_lit");
    return "{" + std::to_string(B.step_a) + ", " + std::to_string(B.path_off) + ", " +
           std::to_string(B.path_len) + ", " + std::to_string(B.ent_first) + ", " +
           std::to_string(B.ent_count) + ", " + std::to_string(B.link) + ", " +
           std::to_string(B.anc_lo) + "u, " + std::to_string(B.anc_hi) + "u, " +
           std::to_string(B.slot_a) + ", " + lit(B.ra) + ", " + lit(B.rqa) + ", " + lit(B.pad) + "}";
}

std::string entry_lit(const EntryRec &E) {
    static_assert(sizeof(EntryRec) == 64, "EntryRec fields changed: update entry_lit");
    return "{" + lit(E.x) + ", " + lit(E.y) + ", " + lit(E.z) + ", " + lit(E.r) + ", " +
           std::to_string(E.mask) + "u, " + lit(E.gate2) + ", " + lit(E.nhr2) + ", " + lit(E.pad) +
           ", " + lits(E.rr, kSpl) + "}";
}

template <class T, class F>
std::string array_lit(const char *type, const char *name, const std::vector<T> &v, F &&one) {
    std::string o = "    static constexpr " + std::string(type) + " " + name + "[" +
                    std::to_string(std::max<size_t>(v.size(), 1)) + "] = {\n";
    if (v.empty()) o += "        " + one(T{}) + ",\n";   // a zero-length array is not C++
    for (const T &x : v) o += "        " + one(x) + ",\n";
    return o + "    };\n";
}

std::string spec_source(const vk_robot_s &r) {
    std::string o = "// robot-specialised persistent edge kernels (generated)\n#include \"vk_walk.hpp\"\n"
                    "namespace vk_spec_robot {\nusing namespace vk;\nstruct R {\n";
    o += "    static constexpr int dof = " + std::to_string(r.dof) + ";\n";
    o += "    static constexpr int n_steps = " + std::to_string(r.steps.size()) + ";\n";
    o += array_lit("StepRec", "steps", r.steps, step_lit);
    o += array_lit("BlockRec", "blocks", r.blocks, block_lit);
    o += array_lit("EntryRec", "entries", r.entries, entry_lit);
    o += array_lit("JointRec", "path_recs", r.path_recs, joint_lit);
    o += "    static constexpr float4 spheres[" + std::to_string(std::max<size_t>(r.spheres.size(), 1)) +
         "] = {\n";
    if (r.spheres.empty()) o += "        {0, 0, 0, 0},\n";
    for (const float4 &x : r.spheres) {
        const float v[4] = {x.x, x.y, x.z, x.w};
        o += "        float4" + lits(v, 4) + ",\n";
    }
    o += "    };\n};\n}  // namespace vk_spec_robot\n";
    o += "#define VK_SPEC_EDGES(NAME, STAGE, COUNT)                                              \\\n"
         "    extern \"C\" __global__ void __launch_bounds__(1024)                                  \\\n"
         "        __attribute__((amdgpu_waves_per_eu(4, 8)))                                      \\\n"
         "        NAME(vk::RobotDev rb, vk::EnvDev ed, const float4 *__restrict__ env_rec,         \\\n"
         "             vk::EdgeSrc src, int64_t n_edges, float res, uint8_t *__restrict__ out,      \\\n"
         "             unsigned long long *__restrict__ queue, int chunk,                          \\\n"
         "             unsigned long long *__restrict__ flops, int cf, int parts, int tparts) {    \\\n"
         "        vk::validate_edges_body<STAGE, COUNT, true>(vk::SpecProg<vk_spec_robot::R>{rb}, ed,\\\n"
         "                                              env_rec, src, n_edges, res, out, queue,    \\\n"
         "                                              chunk, flops, cf, parts, tparts);          \\\n"
         "    }\n";
    for (int c = 0; c < 2; ++c)
        for (int m = 0; m < 3; ++m)
            o += "VK_SPEC_EDGES(vk_spec_edges" + std::string(c ? "_counted_" : "_") + std::to_string(m) +
                 ", " + std::to_string(m) + ", " + (c ? "true" : "false") + ")\n";
    return o;
}

// FNV-1a 64-bit of a string (the code-object cache key)
uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

// Compile the robot's source for `arch` (or take the code object from cache_dir); returns the
// code object.
std::vector<char> spec_compile(const std::string &src, const std::string &arch, const char *cache_dir) {
    std::vector<std::string> opts = {"--offload-arch=" + arch, "-O3", "-std=c++17",
                                     "-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP",
                                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    int n_hdr = 0;
    const char *const *hdr_names = embedded_header_names(&n_hdr);
    const char *const *hdr_text = embedded_header_texts();
    std::string key = src + "|" + arch;
    for (const auto &x : opts) key += "|" + x;
    for (int i = 0; i < n_hdr; ++i) key += std::string("|") + hdr_names[i] + "|" + hdr_text[i];
    char name[64];
    std::snprintf(name, sizeof name, "vk_spec_%016llx.co", (unsigned long long)fnv1a(key));
    const std::string path = cache_dir && *cache_dir ? std::string(cache_dir) + "/" + name : "";
    if (!path.empty()) {
        if (FILE *f = std::fopen(path.c_str(), "rb")) {
            std::vector<char> code;
            char buf[1 << 16];
            size_t got;
            while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) code.insert(code.end(), buf, buf + got);
            std::fclose(f);
            if (!code.empty()) return code;
        }
    }
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, src.c_str(), "vk_spec.hip", n_hdr, hdr_text, hdr_names) !=
        HIPRTC_SUCCESS)
        raise(VK_ERR_HIP, "hiprtcCreateProgram failed");
    std::vector<const char *> o;
    for (const auto &x : opts) o.push_back(x.c_str());
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)o.size(), o.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        raise(VK_ERR_HIP, "specialised kernels did not compile: " + log.substr(0, 2000));
    }
    size_t bytes = 0;
    hiprtcGetCodeSize(prog, &bytes);
    std::vector<char> code(bytes);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (!path.empty()) {                  // best effort: a cache that cannot be written is skipped
        const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
        if (FILE *f = std::fopen(tmp.c_str(), "wb")) {
            const bool ok = std::fwrite(code.data(), 1, code.size(), f) == code.size();
            if (std::fclose(f) == 0 && ok) std::rename(tmp.c_str(), path.c_str());
            else std::remove(tmp.c_str());
        }
    }
    return code;
}
}  // namespace

extern "C" {

vk_status vk_robot_create(const vk_robot_desc *desc, vk_robot *out) {
    return guarded([&] {
        if (!out) raise(VK_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        auto *r = new vk_robot_s();
        try {
            build_robot(desc, r);
        } catch (...) {
            if (r->blob) (void)hipFree(r->blob);   // a failure after the upload
            delete r;
            throw;
        }
        *out = r;
    });
}

vk_status vk_robot_specialize(vk_robot robot, const char *cache_dir) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (robot->module) {
            robot->use_spec = 1;
            return;
        }
        hipDeviceProp_t prop{};
        hip_check(hipGetDeviceProperties(&prop, robot->device), "hipGetDeviceProperties");
        const std::vector<char> code = spec_compile(spec_source(*robot), prop.gcnArchName, cache_dir);
        int cur = 0;
        hip_check(hipGetDevice(&cur), "hipGetDevice");
        if (cur != robot->device) hip_check(hipSetDevice(robot->device), "hipSetDevice");
        hipModule_t mod = nullptr;
        hipError_t err = hipModuleLoadData(&mod, code.data());
        SpecEdgeKernels K;
        for (int m = 0; m < 3 && err == hipSuccess; ++m) {
            const std::string e = "vk_spec_edges_" + std::to_string(m), c = "vk_spec_edges_counted_" + std::to_string(m);
            err = hipModuleGetFunction(&K.edges[m], mod, e.c_str());
            if (err == hipSuccess) err = hipModuleGetFunction(&K.counted[m], mod, c.c_str());
        }
        if (err != hipSuccess && mod) (void)hipModuleUnload(mod);
        if (cur != robot->device) (void)hipSetDevice(cur);
        hip_check(err, "loading the specialised kernels");
        robot->module = mod;
        robot->spec = K;
        robot->use_spec = 1;
    });
}

vk_status vk_robot_use_specialized(vk_robot robot, int32_t on) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (on && !robot->module) raise(VK_ERR_INVALID_ARG, "the robot has not been specialised");
        robot->use_spec = on ? 1 : 0;
    });
}

int32_t vk_robot_is_specialized(vk_robot robot) { return robot ? robot->use_spec.load() : -1; }

int64_t vk_robot_spec_source(const vk_robot_desc *desc, char *buf, int64_t cap) {
    int64_t len = -1;
    const vk_status st = guarded([&] {
        vk_robot_s r;
        build_robot(desc, &r, false);
        const std::string src = spec_source(r);
        len = (int64_t)src.size() + 1;
        if (buf && cap > 0) {
            const size_t n = (size_t)std::min<int64_t>(cap - 1, (int64_t)src.size());
            std::memcpy(buf, src.data(), n);
            buf[n] = '\0';
        }
    });
    return st == VK_OK ? len : -1;
}

vk_status vk_robot_destroy(vk_robot robot) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (robot->module) (void)hipModuleUnload(robot->module);
        hipError_t err = hipFree(robot->blob);
        delete robot;
        hip_check(err, "hipFree");
    });
}

int64_t vk_edge_states(const float *qa, const float *qb, int32_t dof, float resolution) {
    if (!qa || !qb || dof < 1 || dof > kMaxDof || !(resolution > 0.0f && std::isfinite(resolution)))
        return -1;
    double L = 0.0;
    for (int j = 0; j < dof; ++j) {
        if (!std::isfinite(qa[j]) || !std::isfinite(qb[j])) return -1;
        L = std::max(L, std::fabs((double)qb[j] - (double)qa[j]));
    }
    const double n = std::ceil(L / (double)resolution) + 1.0;
    return n < 2.0 ? 2 : (n > 2147483647.0 ? 2147483647 : (int64_t)n);
}

int32_t vk_robot_dof(vk_robot robot) { return robot ? robot->dof : -1; }
int32_t vk_robot_n_spheres(vk_robot robot) { return robot ? robot->n_spheres : -1; }

vk_status vk_env_create(const vk_env_desc *desc, vk_env *out) {
    return guarded([&] {
        if (!out) raise(VK_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        auto *e = new vk_env_s();
        try {
            build_env(desc, e);
        } catch (...) {
            if (e->blob) (void)hipFree(e->blob);   // a failure after the upload (grid record)
            delete e;
            throw;
        }
        *out = e;
    });
}

int64_t vk_env_describe(const vk_env_desc *desc, int64_t *out, int32_t n_out) {
    int64_t bytes = -1;
    const vk_status st = guarded([&] {
        if (n_out < 0 || (n_out > 0 && !out)) raise(VK_ERR_INVALID_ARG, "vk_env_describe: bad output");
        vk_env_s e;
        build_env(desc, &e, false);
        const int64_t v[7] = {e.dev.n_sph, e.dev.n_cap, e.dev.n_cyl, e.dev.n_box, e.n_points,
                              (int64_t)e.dev.n_vox, e.n_vlist};
        const int64_t more[2] = {(int64_t)e.dev.n_cells, e.n_field};
        for (int i = 0; i < n_out && i < 9; ++i) out[i] = i < 7 ? v[i] : more[i - 7];
        bytes = (int64_t)e.host_bytes;
    });
    return st == VK_OK ? bytes : -1;
}

vk_status vk_env_destroy(vk_env env) {
    return guarded([&] {
        if (!env) raise(VK_ERR_INVALID_ARG, "env handle is NULL");
        hipError_t err = hipFree(env->blob);
        delete env;
        hip_check(err, "hipFree");
    });
}

vk_status fk_spheres(vk_robot robot, const float *q, int64_t n, int64_t ldq, float *centres,
                     int64_t ldc, void *stream) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        check_batch(n, ldq, q, centres, "fk_spheres");
        if (ldc < n) raise(VK_ERR_SHAPE, "fk_spheres: ldc < n");
        if (n == 0 || robot->n_spheres == 0) return;
        hip_check(launch_fk_spheres(robot->dev, q, n, ldq, centres, ldc, (hipStream_t)stream),
                  "fk_spheres launch");
    });
}

// The walk's tests in walk order: each link step's environment part, then its self blocks (the
// kernels number them so; blocks are numbered across steps in step order).
static int n_tests(const vk_robot_s &r) { return (int)(r.steps.size() + r.blocks.size()); }

// Number of the first test of link step st (n_tests for st past the last step).
static int step_test(const vk_robot_s &r, int st) {
    return st >= (int)r.steps.size() ? n_tests(r) : st + r.steps[st].blk_first;
}

// Test ranges for a state batch too small to fill the chip (fewer than eight waves per CU): the
// walk's tests split into contiguous ranges of about equal work (an environment part weighs 4,
// a self block 1 plus its entries), as many as keep the split batch within 16 waves per CU, at
// most one per test and kMaxRanges in all.  Each range's waves also pose the steps before it,
// so the split costs work; a batch this small is bound by the latency of one wave's walk, which
// the split shortens.  The robot's max_ranges setting overrides the count (0 or 1: never
// split).
StepRanges state_ranges(const vk_robot_s &r, int64_t n) {
    StepRanges R{};
    const int I = n_tests(r);
    R.n = 1;
    R.b[0] = 0;
    R.b[1] = I;
    const int setting = r.max_ranges.load();
    const int64_t waves = (n + kWave - 1) / kWave;
    int T;
    if (setting < 0) {
        const int64_t n_cu = device_info(r.device).n_cu;
        T = (int)std::min<int64_t>(kMaxRanges, 16 * n_cu / waves);
    } else {
        T = std::min(setting, kMaxRanges);
    }
    T = std::min(T, I);
    if (T <= 1) return R;
    std::vector<double> w;
    w.reserve(I);
    double total = 0.0;
    for (const StepRec &st : r.steps) {
        w.push_back(st.sph_count > 0 ? 4.0 : 1.0);
        for (int b = st.blk_first; b < st.blk_first + st.blk_count; ++b)
            w.push_back(1.0 + r.blocks[b].ent_count);
    }
    for (double x : w) total += x;
    // range y ends after the first test where the running weight reaches (y + 1) / T of the
    // total, leaving at least one test for every later range
    int y = 0;
    double cum = 0.0;
    for (int i = 0; i < I && y < T - 1; ++i) {
        cum += w[i];
        const int left = I - (i + 1);
        if ((cum >= total * (y + 1) / T && left >= T - 1 - y) || left == T - 1 - y) R.b[++y] = i + 1;
    }
    R.n = y + 1;
    R.b[R.n] = I;
    return R;
}

// Test ranges of an edge batch of `waves` one-wave items (edges times rake parts): a batch of
// at most one wave per two CUs splits each edge's walk into ranges of its tests, about one
// wave per two CUs in all (at most one per test and kMaxRanges); the robot's edge_ranges
// setting overrides the count (0 or 1: never split).  The ranges of the edge kernels are of
// equal test count.  Edges are cheaper than states to split wrongly (a short edge's walk is a
// few states), so the automatic split is reserved for a few dozen edges, where one walk's
// latency is the launch: one full-length 7-DoF edge took 61 us unsplit and 44 us split.
static int edge_test_ranges(const vk_robot_s &r, int64_t waves) {
    const int setting = r.edge_ranges.load();
    int64_t T;
    if (setting < 0)
        T = waves > 0 ? (int64_t)device_info(r.device).n_cu / (2 * waves) : 1;
    else
        T = setting;
    T = std::min<int64_t>(std::min<int64_t>(T, kMaxRanges), n_tests(r));
    return T < 2 ? 1 : (int)T;
}

vk_status validate_states(vk_robot robot, vk_env env, const float *q, int64_t n, int64_t ldq,
                          uint8_t *collide, void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, collide, "validate_states");
        if (n == 0) return;
        hipStream_t s = (hipStream_t)stream;
        const int split = step_test(*robot, states_split(robot->dev, n, robot->split_num.load(),
                                                         robot->split_den.load()));
        void *scratch =
            split > 0 ? workspace_for(s, states_scratch_bytes(n), "validate_states").scratch : nullptr;
        const StepRanges ranges = state_ranges(*robot, n);
        hip_check(launch_validate_states(robot->dev,
                                         env_for_launch(env, walk_lds_bytes(robot->dev, walk_block(robot->dev, 256))), q, n,
                                         ldq, collide, split, scratch, s, &ranges),
                  "validate_states launch");
    });
}

vk_status validate_states_noalloc(vk_robot robot, vk_env env, const float *q, int64_t n,
                                  int64_t ldq, uint8_t *collide, void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, collide, "validate_states_noalloc");
        if (n > noalloc_max_states())
            raise(VK_ERR_SHAPE, "validate_states_noalloc: n above its maximum of " +
                                    std::to_string(noalloc_max_states()) + " states");
        if (n == 0) return;
        // the two-pass schedule: the robot's split, else half of its link steps
        int split = states_split(robot->dev, n, robot->split_num.load(), robot->split_den.load());
        if (split == 0) split = states_split(robot->dev, n, 1, 2);
        split = step_test(*robot, split);
        void *scratch = nullptr;
        if (split > 0) hip_check(noalloc_scratch(&scratch), "validate_states_noalloc scratch");
        hip_check(launch_validate_states(robot->dev,
                                         env_for_launch(env, walk_lds_bytes(robot->dev, walk_block(robot->dev, 256))), q, n,
                                         ldq, collide, split, scratch, (hipStream_t)stream),
                  "validate_states_noalloc launch");
    });
}

static void check_edge_inputs(vk_robot robot, vk_env env, const float *qa, const float *qb,
                              const int32_t *n_states, int64_t n_edges, float resolution) {
    check_pair(robot, env);
    if (n_edges < 0) raise(VK_ERR_INVALID_ARG, "n_edges < 0");
    if (n_edges > 0 && (!qa || !qb)) raise(VK_ERR_INVALID_ARG, "NULL edge array");
    if (n_edges >= (int64_t(1) << 31) - (int64_t(1) << 24)) raise(VK_ERR_SHAPE, "too many edges");
    if (!n_states && !(resolution > 0.0f && std::isfinite(resolution)))
        raise(VK_ERR_INVALID_ARG, "resolution must be finite and > 0");
}

static void check_edges(vk_robot robot, vk_env env, const float *qa, const float *qb,
                        const int32_t *n_states, int64_t n_edges, float resolution,
                        uint8_t *collide) {
    check_edge_inputs(robot, env, qa, qb, n_states, n_edges, resolution);
    if (n_edges > 0 && !collide) raise(VK_ERR_INVALID_ARG, "NULL edge array");
}

// A clean slot of the queue ring of (current device, s) for one launch; `wrapped` is set when
// every slot has been used, and then all of them must be zeroed (in stream order) first.
static int take_queue_slot(hipStream_t s, bool &wrapped) {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws.at(std::make_pair(dev, s));
    wrapped = w.next_slot >= kQueueRing;
    if (wrapped) w.next_slot = 0;
    return w.next_slot++;
}

// Zero the counters of every ring slot with one launch.
static hipError_t zero_queue_ring(unsigned long long *queue, hipStream_t s) {
    KernelNode L;
    fill_node(L, queue, 0ull, kQueueRing * kQueues, kQueueWords);
    L.grid = dim3((kQueueRing * kQueues + kWave - 1) / kWave);
    const hipError_t err = hipLaunchKernel(L.fn, L.grid, L.block, L.args, L.shmem, s);
    return err != hipSuccess ? err : hipGetLastError();
}

// Is `s` being captured into a graph?  (A failed query counts as yes: the launch then takes the
// slot it zeroes itself, which is right either way.)
static bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return cap != hipStreamCaptureStatusNone;
}

static void run_edges(vk_robot robot, vk_env env, const EdgeSrc &src, int64_t n_edges,
                      float resolution, uint8_t *collide, unsigned long long *flops,
                      void *stream) {
    if (n_edges == 0) return;
    hipStream_t s = (hipStream_t)stream;
    const int dev = robot->device;
    const DeviceInfo &di = device_info(dev);
    unsigned long long *const ring = workspace_for(s, 0, "validate_edges").queue;
    int block = robot->edge_block.load();
    const int bpc = robot->edge_bpc.load(), tickets = robot->edge_tickets.load();
    const int parts = robot->edge_parts.load();
    const int tparts = flops ? 1 : edge_test_ranges(*robot, n_edges * parts);
    // a workgroup's per-wave caches must fit the LDS: smaller workgroups for large robots
    while (block > kWave && walk_lds_bytes(robot->dev, block) > di.max_lds) block -= kWave;
    // a batch too small to give every CU a workgroup of this size (planner rounds of a few
    // thousand edges) is spread over more CUs in smaller workgroups of at least four waves:
    // such launches are bound by the latency of one walk, not by throughput
    const int64_t items = n_edges * parts * tparts;
    if (items < (int64_t)di.n_cu * (block / kWave)) {
        const int64_t waves = std::max<int64_t>(4, (items + di.n_cu - 1) / di.n_cu);
        block = (int)std::min<int64_t>(block, waves * kWave);
    }
    const int64_t want = (items + block / kWave - 1) / (block / kWave);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)di.n_cu * bpc));
    // edges split over several waves (and the specialised kernels, built in that form) store
    // only the 1s: their flags are zeroed with the queue reset
    const bool spec = robot->use_spec.load() && robot->module;
    const bool multi = spec || parts > 1 || tparts > 1;
    unsigned long long *queue = nullptr;
    if (multi || stream_capturing(s)) {
        queue = ring + (size_t)kQueueRing * kQueueSlotWords;
        hip_check(launch_reset_queue(queue, s, multi ? collide : nullptr, n_edges), "queue reset");
    } else {
        bool wrapped = false;
        const int slot = take_queue_slot(s, wrapped);
        if (wrapped) hip_check(zero_queue_ring(ring, s), "queue ring reset");
        queue = ring + (size_t)slot * kQueueSlotWords;
    }
    const EnvDev ed = env_for_launch(env, walk_lds_bytes(robot->dev, block));
    if (spec)
        hip_check(launch_validate_edges_spec(robot->spec, robot->dev, ed, src, n_edges, resolution,
                                             collide, queue, grid, block, tickets, parts, tparts,
                                             s, flops),
                  "validate_edges launch (specialised)");
    else
        hip_check(launch_validate_edges(robot->dev, ed, src, n_edges, resolution, collide, queue,
                                        grid, block, tickets, parts, tparts, s, flops),
                  "validate_edges launch");
}

vk_status validate_edges(vk_robot robot, vk_env env, const float *qa, const float *qb,
                         const int32_t *n_states, int64_t n_edges, float resolution,
                         uint8_t *collide, void *stream) {
    return guarded([&] {
        check_edges(robot, env, qa, qb, n_states, n_edges, resolution, collide);
        run_edges(robot, env, EdgeSrc{qa, qb, nullptr, 0, n_states}, n_edges, resolution, collide,
                  nullptr, stream);
    });
}

vk_status validate_edges_indexed(vk_robot robot, vk_env env, const float *nodes, int64_t n_nodes,
                                 const int32_t *pairs, const int32_t *n_states, int64_t n_edges,
                                 float resolution, uint8_t *collide, void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        if (n_nodes < 0 || n_edges < 0) raise(VK_ERR_INVALID_ARG, "n_nodes or n_edges < 0");
        if (n_edges > 0 && (!pairs || !collide)) raise(VK_ERR_INVALID_ARG, "NULL pair or flag array");
        if (n_edges > 0 && n_nodes > 0 && !nodes) raise(VK_ERR_INVALID_ARG, "NULL node array");
        if (n_edges >= (int64_t(1) << 31) - (int64_t(1) << 24)) raise(VK_ERR_SHAPE, "too many edges");
        if (!n_states && !(resolution > 0.0f && std::isfinite(resolution)))
            raise(VK_ERR_INVALID_ARG, "resolution must be finite and > 0");
        run_edges(robot, env, EdgeSrc{nodes, nodes, pairs, n_nodes, n_states}, n_edges, resolution,
                  collide, nullptr, stream);
    });
}

vk_status validate_edges_counted(vk_robot robot, vk_env env, const float *qa, const float *qb,
                                 const int32_t *n_states, int64_t n_edges, float resolution,
                                 uint8_t *collide, uint64_t *flops, void *stream) {
    return guarded([&] {
        if (!flops) raise(VK_ERR_INVALID_ARG, "flops is NULL");
        check_edges(robot, env, qa, qb, n_states, n_edges, resolution, collide);
        run_edges(robot, env, EdgeSrc{qa, qb, nullptr, 0, n_states}, n_edges, resolution, collide,
                  reinterpret_cast<unsigned long long *>(flops), stream);
    });
}

vk_status validate_edges_per_edge(vk_robot robot, vk_env env, const float *qa, const float *qb,
                                  const int32_t *n_states, int64_t n_edges, float resolution,
                                  uint8_t *collide, void *stream) {
    return guarded([&] {
        check_edges(robot, env, qa, qb, n_states, n_edges, resolution, collide);
        hipStream_t s = (hipStream_t)stream;
        const EnvDev ed = env_for_launch(env, walk_lds_bytes(robot->dev, kWave));
        for (int64_t e = 0; e < n_edges; ++e)
            hip_check(launch_validate_edge_one(robot->dev, ed, EdgeSrc{qa, qb, nullptr, 0, n_states},
                                               e, resolution, collide, s),
                      "validate_edges_per_edge launch");
    });
}

vk_status vk_knn(const float *x, int64_t n, int32_t dim, int32_t k, int32_t *idx, float *dist2,
                 void *stream) {
    return guarded([&] {
        if (n < 0 || dim < 1 || dim > kMaxDof) raise(VK_ERR_INVALID_ARG, "vk_knn: bad n or dim");
        if (k < 1 || k > 32) raise(VK_ERR_UNSUPPORTED, "vk_knn: k must be in [1, 32]");
        if (n == 0) return;
        if (!x || !idx || !dist2) raise(VK_ERR_INVALID_ARG, "vk_knn: NULL array");
        if (n >= (int64_t(1) << 31) / 32) raise(VK_ERR_SHAPE, "vk_knn: too many samples");
        hipStream_t s = (hipStream_t)stream;
        void *ws = workspace_for(s, knn_workspace_bytes(n, k), "vk_knn").scratch;
        hip_check(launch_knn(x, n, dim, k, idx, dist2, ws, s), "vk_knn launch");
    });
}

vk_status vk_knn_pairs(const int32_t *idx, int64_t n, int32_t k, int32_t *pairs, void *stream) {
    return guarded([&] {
        if (n < 0 || k < 1) raise(VK_ERR_INVALID_ARG, "vk_knn_pairs: bad n or k");
        if (n == 0) return;
        if (!idx || !pairs) raise(VK_ERR_INVALID_ARG, "vk_knn_pairs: NULL array");
        if (n >= (int64_t(1) << 31) / k) raise(VK_ERR_SHAPE, "vk_knn_pairs: too many slots");
        hip_check(launch_knn_pairs(idx, n, k, pairs, (hipStream_t)stream), "vk_knn_pairs launch");
    });
}

static void check_trees(int32_t cap, int32_t dof, int64_t nq) {
    if (cap < 1 || dof < 1 || dof > kMaxDof || nq < 0)
        raise(VK_ERR_INVALID_ARG, "tree call: bad capacity, dof or query count");
    if (nq >= (int64_t(1) << 31) || (int64_t)cap * dof >= (int64_t(1) << 31))
        raise(VK_ERR_SHAPE, "tree call: sizes too large");
}

vk_status vk_tree_nearest(const float *nodes, const int32_t *sizes, int32_t cap, int32_t dof,
                          int64_t nq, const float *targets, const uint8_t *active, int32_t *near,
                          void *stream) {
    return guarded([&] {
        check_trees(cap, dof, nq);
        if (nq == 0) return;
        if (!nodes || !sizes || !targets || !near) raise(VK_ERR_INVALID_ARG, "vk_tree_nearest: NULL array");
        hip_check(launch_tree_nearest(nodes, sizes, cap, dof, nq, targets, active, near,
                                      (hipStream_t)stream),
                  "vk_tree_nearest launch");
    });
}

vk_status vk_tree_steer(const float *nodes, int32_t cap, int32_t dof, int64_t nq,
                        const int32_t *near, const float *targets, float step, float *qnew,
                        uint8_t *reached, void *stream) {
    return guarded([&] {
        check_trees(cap, dof, nq);
        if (!(step > 0.0f && std::isfinite(step))) raise(VK_ERR_INVALID_ARG, "vk_tree_steer: step must be > 0");
        if (nq == 0) return;
        if (!nodes || !near || !targets || !qnew || !reached)
            raise(VK_ERR_INVALID_ARG, "vk_tree_steer: NULL array");
        hip_check(launch_tree_steer(nodes, cap, dof, nq, near, targets, step, qnew, reached,
                                    (hipStream_t)stream),
                  "vk_tree_steer launch");
    });
}

vk_status vk_tree_append(float *nodes, int32_t *parents, int32_t *sizes, int32_t cap, int32_t dof,
                         int64_t nq, const float *qnew, const int32_t *near, const uint8_t *ok,
                         int32_t *added, void *stream) {
    return guarded([&] {
        check_trees(cap, dof, nq);
        if (nq == 0) return;
        if (!nodes || !parents || !sizes || !qnew || !near || !ok || !added)
            raise(VK_ERR_INVALID_ARG, "vk_tree_append: NULL array");
        hip_check(launch_tree_append(nodes, parents, sizes, cap, dof, nq, qnew, near, ok, added,
                                     (hipStream_t)stream),
                  "vk_tree_append launch");
    });
}

vk_status vk_rrt_extend(const float *nodes, const int32_t *sizes, int32_t cap, int32_t dof,
                        int64_t nq, const float *targets, const uint8_t *active, float step,
                        float *qnear, float *qnew, int32_t *near, uint8_t *reached,
                        void *stream) {
    return guarded([&] {
        check_trees(cap, dof, nq);
        if (!(step > 0.0f && std::isfinite(step))) raise(VK_ERR_INVALID_ARG, "vk_rrt_extend: step must be > 0");
        if (nq == 0) return;
        if (!nodes || !sizes || !targets || !active || !qnear || !qnew || !near || !reached)
            raise(VK_ERR_INVALID_ARG, "vk_rrt_extend: NULL array");
        hip_check(launch_rrt_extend(nodes, sizes, cap, dof, nq, targets, active, step, qnear, qnew,
                                    near, reached, (hipStream_t)stream),
                  "vk_rrt_extend launch");
    });
}

vk_status vk_rrt_commit(float *nodes, int32_t *parents, int32_t *sizes, int32_t cap, int32_t dof,
                        int64_t nq, const float *qnew, const int32_t *near, const uint8_t *reached,
                        const uint8_t *flags, uint8_t *going, int32_t *added,
                        const int32_t *from_added, int64_t *meet_this, int64_t *meet_from,
                        uint8_t *solved, uint64_t *edges, void *stream) {
    return guarded([&] {
        check_trees(cap, dof, nq);
        if (nq == 0) return;
        if (!nodes || !parents || !sizes || !qnew || !near || !reached || !flags || !going ||
            !added || !edges)
            raise(VK_ERR_INVALID_ARG, "vk_rrt_commit: NULL array");
        if (from_added && (!meet_this || !meet_from || !solved))
            raise(VK_ERR_INVALID_ARG, "vk_rrt_commit: from_added needs meet_this, meet_from and solved");
        hip_check(launch_rrt_commit(nodes, parents, sizes, cap, dof, nq, qnew, near, reached, flags,
                                    going, added, from_added, meet_this, meet_from, solved, edges,
                                    (hipStream_t)stream),
                  "vk_rrt_commit launch");
    });
}

static void check_paths(int64_t P, int32_t M, int32_t K, int32_t dof) {
    if (P < 0 || M < 1 || K < 1 || K > 64 || dof < 1 || dof > kMaxDof)
        raise(VK_ERR_INVALID_ARG, "shortcut: need P >= 0, M >= 1, 1 <= K <= 64, 1 <= dof <= 64");
    if (P * (int64_t)M >= (int64_t(1) << 31) || P * (int64_t)K >= (int64_t(1) << 31) - (int64_t(1) << 24))
        raise(VK_ERR_SHAPE, "shortcut: too many waypoints or candidates");
}

vk_status vk_shortcut_propose(const int32_t *lens, int64_t n_paths, int32_t max_len, int32_t k,
                              const uint32_t *rnd, int32_t *pairs, void *stream) {
    return guarded([&] {
        check_paths(n_paths, max_len, k, 1);
        if (n_paths == 0) return;
        if (!lens || !rnd || !pairs) raise(VK_ERR_INVALID_ARG, "vk_shortcut_propose: NULL array");
        hip_check(launch_shortcut_propose(lens, n_paths, max_len, k, rnd, pairs, (hipStream_t)stream),
                  "vk_shortcut_propose launch");
    });
}

vk_status vk_shortcut_apply(float *paths, int32_t *lens, int64_t n_paths, int32_t max_len,
                            int32_t dof, int32_t k, const int32_t *pairs, const uint8_t *collide,
                            uint8_t *accepted, void *stream) {
    return guarded([&] {
        check_paths(n_paths, max_len, k, dof);
        if (n_paths == 0) return;
        if (!paths || !lens || !pairs || !collide)
            raise(VK_ERR_INVALID_ARG, "vk_shortcut_apply: NULL array");
        hip_check(launch_shortcut_apply(paths, lens, n_paths, max_len, dof, k, pairs, collide,
                                        accepted, (hipStream_t)stream),
                  "vk_shortcut_apply launch");
    });
}

vk_status penetration_cost_fwd(vk_robot robot, vk_env env, const float *q, int64_t n,
                               int64_t ldq, float *cost, void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, cost, "penetration_cost_fwd");
        if (n == 0) return;
        hip_check(launch_cost_fwd(robot->dev,
                                  env_for_launch(env, walk_lds_bytes(robot->dev, walk_block(robot->dev, 256))),
                                  q, n, ldq, cost,
                                  (hipStream_t)stream),
                  "penetration_cost_fwd launch");
    });
}

// Workgroup size of the adjoint with its force slots in LDS: three waves (the slots make the
// LDS the limit, and three 3-wave workgroups of the 7-DoF robot fit a CU where only two 4-wave
// ones do), fewer for robots whose slots do not fit.
static int cost_lds_block(const vk_robot_s &r) {
    const DeviceInfo &di = device_info(r.device);
    int block = 192;
    while (block > 64 && cost_bwd_slot_bytes(r.dev, block, 0) > di.max_lds) block -= 64;
    return block;
}

// Global-memory scratch for the adjoint's force slots at n states, 0 when they stay in LDS.
// The LDS holds the adjoint to a few waves per CU (the slots are 24 bytes per link and state); a
// batch that needs more than one round of those waves runs faster with the slots in global
// memory and four waves per SIMD (262,144 7-DoF states: 175 -> 148 us), a smaller one slower
// (the slots' reads and writes then lengthen the one round: 131,072 states 109 -> 133 us).
static size_t cost_scratch_bytes(const vk_robot_s &r, int64_t n) {
    const DeviceInfo &di = device_info(r.device);
    const int64_t waves = (n + kWave - 1) / kWave;
    const int64_t lds_waves = (int64_t)cost_bwd_lds_waves_per_cu(r.dev, cost_lds_block(r)) * di.n_cu;
    if (waves <= lds_waves) return 0;
    return cost_bwd_global_slot_bytes(r.dev, n, walk_block(r.dev, 256));
}

// the adjoint launch shared by penetration_cost_bwd and penetration_cost_fwd_grad
static void run_cost_bwd(vk_robot robot, vk_env env, const float *q, int64_t n, int64_t ldq,
                         const float *grad_cost, float *grad_q, int64_t ldg, float *cost,
                         void *stream) {
    const DeviceInfo &di = device_info(robot->device);
    // the slots in global memory when the batch is large enough and the stream's workspace
    // holds them (vk_reserve_cost), else in LDS: the same results either way
    const size_t need = cost_scratch_bytes(*robot, n);
    float *gslots = nullptr;
    if (need > 0) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(current_device(), (hipStream_t)stream));
        if (it != g_ws.end() && it->second.scratch_bytes >= need)
            gslots = static_cast<float *>(it->second.scratch);
    }
    if (gslots) {
        const int gblock = walk_block(robot->dev, 256);
        hip_check(launch_cost_bwd(robot->dev, env_for_launch(env, walk_lds_bytes(robot->dev, gblock)),
                                  q, n, ldq, grad_cost, grad_q, ldg, gblock, (hipStream_t)stream,
                                  cost, gslots),
                  "penetration cost adjoint launch");
        return;
    }
    const int block = cost_lds_block(*robot);
    const size_t slots = cost_bwd_slot_bytes(robot->dev, block, 0);
    if (slots > di.max_lds) raise(VK_ERR_UNSUPPORTED, "robot too large for the backward kernel");
    hip_check(launch_cost_bwd(robot->dev, env_for_launch(env, slots), q, n, ldq, grad_cost, grad_q,
                              ldg, block, (hipStream_t)stream, cost),
              "penetration cost adjoint launch");
}

vk_status penetration_cost_bwd(vk_robot robot, vk_env env, const float *q, int64_t n,
                               int64_t ldq, const float *grad_cost, float *grad_q, int64_t ldg,
                               void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, grad_q, "penetration_cost_bwd");
        if (n > 0 && !grad_cost) raise(VK_ERR_INVALID_ARG, "grad_cost is NULL");
        if (ldg < n) raise(VK_ERR_SHAPE, "penetration_cost_bwd: ldg < n");
        if (n == 0) return;
        run_cost_bwd(robot, env, q, n, ldq, grad_cost, grad_q, ldg, nullptr, stream);
    });
}

vk_status penetration_cost_fwd_grad(vk_robot robot, vk_env env, const float *q, int64_t n,
                                    int64_t ldq, float *cost, float *grad_q, int64_t ldg,
                                    void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, grad_q, "penetration_cost_fwd_grad");
        if (n > 0 && !cost) raise(VK_ERR_INVALID_ARG, "cost is NULL");
        if (ldg < n) raise(VK_ERR_SHAPE, "penetration_cost_fwd_grad: ldg < n");
        if (n == 0) return;
        run_cost_bwd(robot, env, q, n, ldq, nullptr, grad_q, ldg, cost, stream);
    });
}

vk_status vk_edge_batch_create(const vk_robot *robots, int32_t n_robots, const vk_env *envs,
                               int32_t n_envs, const vk_edge_set *sets, int32_t n_sets,
                               float resolution, int32_t block_threads, int32_t blocks_per_cu,
                               vk_edge_batch *out) {
    return guarded([&] {
        if (!out) raise(VK_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (n_robots < 1 || n_envs < 1 || n_sets < 0 || !robots || !envs || (n_sets && !sets))
            raise(VK_ERR_INVALID_ARG, "robots, envs and sets must be non-empty arrays");
        if (!(resolution > 0.0f && std::isfinite(resolution)))
            raise(VK_ERR_INVALID_ARG, "resolution must be finite and > 0");
        if (block_threads == 0 && blocks_per_cu == 0) {
            block_threads = kDefaultEdgeBlock;
            blocks_per_cu = kDefaultEdgeBpc;
        }
        check_launch(block_threads, blocks_per_cu, kDefaultTickets);
        for (int i = 0; i < n_robots; ++i)
            if (!robots[i]) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        for (int i = 0; i < n_envs; ++i)
            if (!envs[i]) raise(VK_ERR_INVALID_ARG, "env handle is NULL");
        std::vector<BatchSet> recs;
        int64_t total = 0;
        for (int k = 0; k < n_sets; ++k) {
            const vk_edge_set &s = sets[k];
            if (s.robot < 0 || s.robot >= n_robots || s.env < 0 || s.env >= n_envs)
                raise(VK_ERR_INVALID_ARG, "edge set refers to a missing robot or env");
            if (s.n_edges < 0 || s.qa_offset < 0 || s.out_offset < 0)
                raise(VK_ERR_INVALID_ARG, "negative edge-set size or offset");
            if (s.n_edges == 0) continue;
            BatchSet b;
            std::memset(&b, 0, sizeof b);
            b.rb = robots[s.robot]->dev;
            b.env = envs[s.env]->dev;
            b.qa_offset = s.qa_offset;
            b.n_edges = s.n_edges;
            b.out_offset = s.out_offset;
            b.first = total;
            recs.push_back(b);
            total += s.n_edges;
        }
        if (total >= (int64_t(1) << 31) - (int64_t(1) << 24)) raise(VK_ERR_SHAPE, "too many edges");
        auto *bt = new vk_edge_batch_s();
        try {
            bt->device = current_device();
            bt->total = total;
            // the set of every edge (sets in order, each covering its n_edges consecutive edges)
            std::vector<int32_t> edge_set((size_t)std::max<int64_t>(total, 1), 0);
            for (size_t k = 0; k < recs.size(); ++k)
                std::fill(edge_set.begin() + recs[k].first,
                          edge_set.begin() + recs[k].first + recs[k].n_edges, (int32_t)k);
            if (recs.empty()) recs.push_back(BatchSet{});
            Blob bl;
            const size_t o_s = bl.add(recs.data(), recs.size() * sizeof(BatchSet));
            const size_t o_p = bl.add(edge_set.data(), edge_set.size() * sizeof(int32_t));
            bt->blob = bl.upload();
            void *q = nullptr;
            hip_check(hipMalloc(&q, kQueueBytes), "batch queue");
            bt->queue = static_cast<unsigned long long *>(q);
            const BatchSet *d_sets = reinterpret_cast<const BatchSet *>(static_cast<char *>(bt->blob) + o_s);
            const int32_t *d_eset = reinterpret_cast<const int32_t *>(static_cast<char *>(bt->blob) + o_p);
            const DeviceInfo &di = device_info(bt->device);
            int block = block_threads;
            // per wave: link bound centres, and optionally capsule halves and joint values
            int max_slots = 0, max_dof = 0;
            for (const BatchSet &b : recs) {
                max_slots = std::max(max_slots, b.rb.n_slots);
                max_dof = std::max(max_dof, b.rb.dof);
            }
            const int min_floats = step_cache_floats(max_slots, max_dof, 0);
            while (block > kWave && (size_t)(block / kWave) * min_floats * sizeof(float) > di.max_lds)
                block -= kWave;
            if ((size_t)(block / kWave) * min_floats * sizeof(float) > di.max_lds)
                raise(VK_ERR_UNSUPPORTED, "robots too large for the LDS walk cache");
            const int64_t want = (total + block / kWave - 1) / (block / kWave);
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)di.n_cu * blocks_per_cu));
            bt->block = block_threads;
            bt->per_cu = blocks_per_cu;
            // the graph {queue reset -> persistent launch}; run() points the launch's node at
            // the caller's arrays and replays it
            fill_node(bt->reset, bt->queue, 0ull, kQueues, kQueueWords);
            edge_batch_node(bt->launch, d_sets, d_eset, (int)recs.size(), total, resolution,
                            bt->queue, grid, block, kDefaultTickets, max_slots, max_dof);
            hip_check(hipGraphCreate(&bt->graph, 0), "hipGraphCreate");
            const auto params = [](KernelNode &L) {
                hipKernelNodeParams p{};
                p.func = const_cast<void *>(L.fn);
                p.gridDim = L.grid;
                p.blockDim = L.block;
                p.sharedMemBytes = (unsigned)L.shmem;
                p.kernelParams = L.args;
                p.extra = nullptr;
                return p;
            };
            hipGraphNode_t reset = nullptr;
            hipKernelNodeParams pr = params(bt->reset);
            hip_check(hipGraphAddKernelNode(&reset, bt->graph, nullptr, 0, &pr), "graph reset node");
            if (total > 0) {
                hipKernelNodeParams pl = params(bt->launch);
                hip_check(hipGraphAddKernelNode(&bt->walk, bt->graph, &reset, 1, &pl), "graph launch node");
            }
            hip_check(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        } catch (...) {
            if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
            if (bt->graph) (void)hipGraphDestroy(bt->graph);
            if (bt->queue) (void)hipFree(bt->queue);
            if (bt->blob) (void)hipFree(bt->blob);
            delete bt;
            throw;
        }
        *out = bt;
    });
}

vk_status vk_edge_batch_run(vk_edge_batch batch, const float *qa, const float *qb,
                            uint8_t *collide, void *stream) {
    return guarded([&] {
        if (!batch) raise(VK_ERR_INVALID_ARG, "batch handle is NULL");
        if (batch->total > 0) {
            if (!qa || !qb || !collide) raise(VK_ERR_INVALID_ARG, "NULL edge array");
            auto &a = batch->launch.batch;
            if (a.qa != qa || a.qb != qb || a.out != collide) {
                a.qa = qa;
                a.qb = qb;
                a.out = collide;
                hipKernelNodeParams p{};
                p.func = const_cast<void *>(batch->launch.fn);
                p.gridDim = batch->launch.grid;
                p.blockDim = batch->launch.block;
                p.sharedMemBytes = (unsigned)batch->launch.shmem;
                p.kernelParams = batch->launch.args;
                p.extra = nullptr;
                hip_check(hipGraphExecKernelNodeSetParams(batch->exec, batch->walk, &p),
                          "batch arrays update");
            }
        }
        hip_check(hipGraphLaunch(batch->exec, (hipStream_t)stream), "hipGraphLaunch");
    });
}

vk_status vk_edge_batch_destroy(vk_edge_batch batch) {
    return guarded([&] {
        if (!batch) raise(VK_ERR_INVALID_ARG, "batch handle is NULL");
        (void)hipGraphExecDestroy(batch->exec);
        (void)hipGraphDestroy(batch->graph);
        (void)hipFree(batch->queue);
        hipError_t err = hipFree(batch->blob);
        delete batch;
        hip_check(err, "hipFree");
    });
}

vk_status vk_edge_batch_get_launch(vk_edge_batch batch, int32_t *block_threads,
                                   int32_t *blocks_per_cu) {
    return guarded([&] {
        if (!batch) raise(VK_ERR_INVALID_ARG, "batch handle is NULL");
        if (!block_threads || !blocks_per_cu) raise(VK_ERR_INVALID_ARG, "NULL output");
        *block_threads = batch->block;
        *blocks_per_cu = batch->per_cu;
    });
}

// Grow the workspace of (current device, s) to the queue counters and `bytes` of scratch.
static void reserve_workspace(hipStream_t s, size_t bytes) {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws[std::make_pair(dev, s)];
    const bool need_queue = !w.queue, need_scratch = bytes > w.scratch_bytes;
    if (!need_queue && !need_scratch) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        raise(VK_ERR_SHAPE, "vk_reserve: the stream is being captured and its workspace must "
                            "grow; reserve before the capture");
    if (need_queue) {
        void *p = nullptr;
        hip_check(hipMalloc(&p, (kQueueRing + 1) * kQueueBytes), "vk_reserve: queue counters");
        w.queue = static_cast<unsigned long long *>(p);
    }
    if (need_scratch) {
        void *p = nullptr;
        hip_check(hipMalloc(&p, bytes), "vk_reserve: scratch");
        if (w.scratch) w.retired.push_back(w.scratch);   // work or graphs may still use it
        w.scratch = p;
        w.scratch_bytes = bytes;
    }
}

vk_status vk_reserve(void *stream, int64_t max_states, int64_t max_knn_samples, int32_t max_knn_k) {
    return guarded([&] {
        if (max_states < 0 || max_knn_samples < 0 || max_knn_k < 0 || max_knn_k > 32)
            raise(VK_ERR_INVALID_ARG, "vk_reserve: sizes must be >= 0 and max_knn_k <= 32");
        if (max_states >= (int64_t(1) << 31) || max_knn_samples >= (int64_t(1) << 31) / 32)
            raise(VK_ERR_SHAPE, "vk_reserve: sizes too large");
        reserve_workspace((hipStream_t)stream, reserve_bytes(max_states, max_knn_samples, max_knn_k));
    });
}

vk_status vk_reserve_cost(void *stream, vk_robot robot, int64_t max_states) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (max_states < 0) raise(VK_ERR_INVALID_ARG, "vk_reserve_cost: max_states < 0");
        if (max_states >= (int64_t(1) << 31)) raise(VK_ERR_SHAPE, "vk_reserve_cost: max_states too large");
        // the slots of the largest batch that keeps them in global memory; a batch that keeps
        // them in LDS needs none, and for those the queue counters alone are reserved
        reserve_workspace((hipStream_t)stream, cost_scratch_bytes(*robot, max_states));
    });
}

vk_status vk_release(void *stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        const int dev = current_device();
        Workspace w;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_ws.find(std::make_pair(dev, s));
            if (it == g_ws.end()) return;
            w = std::move(it->second);
            g_ws.erase(it);
        }
        hip_check(hipStreamSynchronize(s), "vk_release: stream sync");
        hipError_t err = hipSuccess;
        for (void *p : w.retired) err = err != hipSuccess ? err : hipFree(p);
        if (w.scratch) err = err != hipSuccess ? err : hipFree(w.scratch);
        if (w.queue) err = err != hipSuccess ? err : hipFree(w.queue);
        hip_check(err, "vk_release: hipFree");
    });
}

vk_status vk_robot_set_states_split(vk_robot robot, int32_t num, int32_t den) {
    return guarded([&] {
        if (num < 0 || den < 1 || num >= den) raise(VK_ERR_INVALID_ARG, "need 0 <= num < den");
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        robot->split_num = num;
        robot->split_den = den;
    });
}

vk_status vk_robot_get_states_split(vk_robot robot, int32_t *num, int32_t *den) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (!num || !den) raise(VK_ERR_INVALID_ARG, "NULL output");
        *num = robot->split_num;
        *den = robot->split_den;
    });
}

vk_status vk_robot_set_states_ranges(vk_robot robot, int32_t max_ranges) {
    return guarded([&] {
        if (max_ranges < -1 || max_ranges > kMaxRanges)
            raise(VK_ERR_INVALID_ARG, "max_ranges must be -1 (automatic) or in [0, 32]");
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        robot->max_ranges = max_ranges;
    });
}

vk_status vk_robot_get_states_ranges(vk_robot robot, int32_t *max_ranges) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (!max_ranges) raise(VK_ERR_INVALID_ARG, "NULL output");
        *max_ranges = robot->max_ranges;
    });
}

vk_status vk_robot_set_edge_parts(vk_robot robot, int32_t parts) {
    return guarded([&] {
        if (parts < 1 || parts > 64) raise(VK_ERR_INVALID_ARG, "parts must be in [1, 64]");
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        robot->edge_parts = parts;
    });
}

int32_t vk_robot_get_edge_parts(vk_robot robot) { return robot ? robot->edge_parts.load() : -1; }

vk_status vk_robot_set_edge_ranges(vk_robot robot, int32_t max_ranges) {
    return guarded([&] {
        if (max_ranges < -1 || max_ranges > kMaxRanges)
            raise(VK_ERR_INVALID_ARG, "max_ranges must be -1 (automatic) or in [0, 32]");
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        robot->edge_ranges = max_ranges;
    });
}

int32_t vk_robot_get_edge_ranges(vk_robot robot) { return robot ? robot->edge_ranges.load() : -2; }

vk_status vk_robot_set_edge_launch(vk_robot robot, int32_t block_threads, int32_t blocks_per_cu,
                                   int32_t tickets_per_wave) {
    return guarded([&] {
        if (block_threads == 0 && blocks_per_cu == 0 && tickets_per_wave == 0) {
            block_threads = kDefaultEdgeBlock;
            blocks_per_cu = kDefaultEdgeBpc;
            tickets_per_wave = kDefaultTickets;
        }
        check_launch(block_threads, blocks_per_cu, tickets_per_wave);
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        robot->edge_block = block_threads;
        robot->edge_bpc = blocks_per_cu;
        robot->edge_tickets = tickets_per_wave;
    });
}

vk_status vk_robot_get_edge_launch(vk_robot robot, int32_t *block_threads, int32_t *blocks_per_cu,
                                   int32_t *tickets_per_wave) {
    return guarded([&] {
        if (!robot) raise(VK_ERR_INVALID_ARG, "robot handle is NULL");
        if (!block_threads || !blocks_per_cu || !tickets_per_wave) raise(VK_ERR_INVALID_ARG, "NULL output");
        *block_threads = robot->edge_block;
        *blocks_per_cu = robot->edge_bpc;
        *tickets_per_wave = robot->edge_tickets;
    });
}

vk_status vk_autotune_edges(vk_robot robot, vk_env env, const float *qa, const float *qb,
                            const int32_t *n_states, int64_t n_edges, float resolution,
                            const char *cache_path, int32_t force, void *stream) {
    return guarded([&] {
        check_edge_inputs(robot, env, qa, qb, n_states, n_edges, resolution);
        if (n_edges == 0) return;
        hipStream_t s = (hipStream_t)stream;
        const std::string key = tune_key("edges", robot, env, n_edges);
        TuneCache cache = load_tune_cache(cache_path);
        auto hit = cache.find(key);
        if (!force && hit != cache.end()) {
            const int block = entry_int(hit->second, "block"), bpc = entry_int(hit->second, "per_cu"),
                      tickets = entry_int(hit->second, "tickets");
            const int parts = hit->second.count("parts") ? entry_int(hit->second, "parts") : 1;
            bool valid = parts >= 1 && parts <= 64;
            try {
                check_launch(block, bpc, tickets);
            } catch (const VkError &) {
                valid = false;                 // a damaged entry: time the workload again
            }
            if (valid) {
                robot->edge_block = block;
                robot->edge_bpc = bpc;
                robot->edge_tickets = tickets;
                robot->edge_parts = parts;
                return;
            }
        }
        if (vk_reserve(stream, 0, 0, 0) != VK_OK) raise(VK_ERR_OOM, "autotune workspace: " + g_err);
        uint8_t *flags = nullptr;
        hip_check(hipMalloc(&flags, (size_t)n_edges), "autotune flags");
        std::vector<std::array<double, 4>> results;   // ms, block, per_cu, tickets
        std::vector<std::array<double, 2>> by_parts;  // ms, parts
        try {
            const EdgeSrc src{qa, qb, nullptr, 0, n_states};
            robot->edge_parts = 1;
            for (int block : {64, 128, 256, 512, 1024})
                for (int bpc : {1, 2, 4, 8}) {
                    if (block * bpc > 2048) continue;      // more waves than a CU holds
                    for (int tickets : {4, 8, 16}) {
                        robot->edge_block = block;
                        robot->edge_bpc = bpc;
                        robot->edge_tickets = tickets;
                        const double ms = time_median(s, [&] {
                            run_edges(robot, env, src, n_edges, resolution, flags, nullptr, stream);
                        });
                        results.push_back({ms, (double)block, (double)bpc, (double)tickets});
                    }
                }
            // the fastest few again, interleaved over three rounds, each scored by the median of
            // its rounds: launches a few percent apart are within one round's noise
            std::sort(results.begin(), results.end());
            const size_t n_fin = std::min<size_t>(4, results.size());
            std::vector<std::vector<double>> rounds(n_fin);
            for (int round = 0; round < 3; ++round)
                for (size_t f = 0; f < n_fin; ++f) {
                    robot->edge_block = (int)results[f][1];
                    robot->edge_bpc = (int)results[f][2];
                    robot->edge_tickets = (int)results[f][3];
                    rounds[f].push_back(time_median(s, [&] {
                        run_edges(robot, env, src, n_edges, resolution, flags, nullptr, stream);
                    }));
                }
            size_t win = 0;
            double win_ms = 0.0;
            for (size_t f = 0; f < n_fin; ++f) {
                std::sort(rounds[f].begin(), rounds[f].end());
                if (f == 0 || rounds[f][1] < win_ms) {
                    win = f;
                    win_ms = rounds[f][1];
                }
            }
            const auto best = results[win];
            robot->edge_block = (int)best[1];
            robot->edge_bpc = (int)best[2];
            robot->edge_tickets = (int)best[3];
            by_parts.push_back({win_ms, 1.0});
            for (int parts : {2, 4, 8}) {
                robot->edge_parts = parts;
                by_parts.push_back({time_median(s, [&] {
                                        run_edges(robot, env, src, n_edges, resolution, flags,
                                                  nullptr, stream);
                                    }),
                                    (double)parts});
            }
        } catch (...) {
            robot->edge_parts = 1;
            (void)hipFree(flags);
            throw;
        }
        hip_check(hipFree(flags), "hipFree");
        const auto bp = *std::min_element(by_parts.begin(), by_parts.end());
        robot->edge_parts = (int)bp[1];
        if (cache_path && *cache_path) {
            TuneCache now = load_tune_cache(cache_path);
            now[key] = {{"block", (double)robot->edge_block.load()}, {"per_cu", (double)robot->edge_bpc.load()},
                        {"tickets", (double)robot->edge_tickets.load()}, {"parts", bp[1]}, {"ms", bp[0]}};
            save_tune_cache(cache_path, now);
        }
    });
}

vk_status vk_autotune_states(vk_robot robot, vk_env env, const float *q, int64_t n, int64_t ldq,
                             const char *cache_path, int32_t force, void *stream) {
    return guarded([&] {
        check_pair(robot, env);
        check_batch(n, ldq, q, q, "vk_autotune_states");   // no output array: q stands in
        if (n == 0) return;
        hipStream_t s = (hipStream_t)stream;
        const std::string key = tune_key("states", robot, env, n);
        TuneCache cache = load_tune_cache(cache_path);
        auto hit = cache.find(key);
        if (!force && hit != cache.end()) {
            const int num = entry_int(hit->second, "num"), den = entry_int(hit->second, "den");
            if (num >= 0 && den >= 1 && num < den) {   // else a damaged entry: time it again
                robot->split_num = num;
                robot->split_den = den;
                return;
            }
        }
        if (vk_reserve(stream, n, 0, 0) != VK_OK) raise(VK_ERR_OOM, "autotune workspace: " + g_err);
        uint8_t *flags = nullptr;
        hip_check(hipMalloc(&flags, (size_t)n), "autotune flags");
        std::vector<std::array<double, 3>> results;   // ms, num, den
        try {
            for (const auto &sp : {std::array<int, 2>{0, 1}, {1, 3}, {1, 2}, {2, 3}}) {
                robot->split_num = sp[0];
                robot->split_den = sp[1];
                const double ms = time_median(s, [&] {
                    if (validate_states(robot, env, q, n, ldq, flags, stream) != VK_OK)
                        raise(VK_ERR_HIP, "autotune: " + g_err);
                });
                results.push_back({ms, (double)sp[0], (double)sp[1]});
            }
        } catch (...) {
            (void)hipFree(flags);
            throw;
        }
        hip_check(hipFree(flags), "hipFree");
        const auto best = *std::min_element(results.begin(), results.end());
        robot->split_num = (int)best[1];
        robot->split_den = (int)best[2];
        if (cache_path && *cache_path) {
            TuneCache now = load_tune_cache(cache_path);
            now[key] = {{"num", best[1]}, {"den", best[2]}, {"ms", best[0]}};
            save_tune_cache(cache_path, now);
        }
    });
}

const char *vk_last_error(void) { return g_err.c_str(); }

}  // extern "C"
