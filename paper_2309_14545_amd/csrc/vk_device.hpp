// Device building blocks: per-lane frames, the revolute DH joint update, sphere placement and
// sphere-vs-primitive overlap tests.  One lane holds one configuration; every robot or
// environment value is wave-uniform.
#pragma once
#ifndef __HIPCC_RTC__                 // the runtime compiler provides the HIP device runtime itself
#include <hip/hip_runtime.h>
#endif

#include "vk_types.hpp"

namespace vk {

// Rigid transform held in registers: rotation row-major r[3*i + k], translation p.
struct Frame {
    float r[9];
    float p[3];
};

__device__ __forceinline__ void frame_identity(Frame &T) {
#pragma unroll
    for (int i = 0; i < 9; ++i) T.r[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    T.p[0] = T.p[1] = T.p[2] = 0.0f;
}

// T <- T * M for a fixed mount M (row-major 3x4, wave-uniform).
__device__ __forceinline__ void frame_mount(Frame &T, const float *m) {
    float r[9], p[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r[3 * i + k] = fmaf(T.r[3 * i], m[k], fmaf(T.r[3 * i + 1], m[4 + k], T.r[3 * i + 2] * m[8 + k]));
        p[i] = fmaf(T.r[3 * i], m[3], fmaf(T.r[3 * i + 1], m[7], fmaf(T.r[3 * i + 2], m[11], T.p[i])));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) T.r[i] = r[i];
    T.p[0] = p[0];
    T.p[1] = p[1];
    T.p[2] = p[2];
}

// Values of one joint at q: sine and cosine of the DH angle and the offset along z.  A revolute
// joint turns (angle q + theta_off, offset d); a prismatic joint slides (angle theta_off, whose
// sine and cosine come with the record, offset d + q).
struct JointVal {
    float s, c, d;
};

// Sine and cosine of x (radians) from the hardware sine and cosine of a fraction of a turn.
// x / 2pi = n + f with n an integer and |f| <= 1/2 (Cody and Waite's argument reduction, with
// the period measured in turns): an FMA forms x * hi - n from the exact product, rounded once,
// and a second FMA adds x * lo, the part of 1/2pi that hi (1/2pi rounded to FP32) leaves out.
// f then holds x / 2pi - n to within about an ulp of f plus |x| * 1e-16, and the hardware
// evaluates sin(2 pi f) and cos(2 pi f).
__device__ __forceinline__ void sincos_turns(float x, float &s, float &c) {
    constexpr float kInv2PiHi = 0x1.45f306p-3f;    // 1/2pi rounded to FP32
    constexpr float kInv2PiLo = 0x1.b93910p-28f;   // 1/2pi - kInv2PiHi, rounded
    const float n = rintf(x * kInv2PiHi);
    const float f = fmaf(x, kInv2PiLo, fmaf(x, kInv2PiHi, -n));
    s = __builtin_amdgcn_sinf(f);
    c = __builtin_amdgcn_cosf(f);
}

__device__ __forceinline__ JointVal joint_val(const JointRec &J, float q) {
    JointVal v;
    if (J.prismatic) {
        v.s = J.s_off;
        v.c = J.c_off;
        v.d = J.d + q;
    } else {
        sincos_turns(q + J.theta_off, v.s, v.c);
        v.d = J.d;
    }
    return v;
}

// T <- T * Rz(theta) Tz(d) Tx(a) Rx(alpha): the standard DH link transform (Sec. III-B).
// Column form: c0' = c c0 + s c1, c1' = -s c0 + c c1, p' = p + d c2 + a c0', then the twist
// mixes c1' and c2.  Twists of 0 and +-90 degrees are folded (no multiplies); the twist is
// wave-uniform, so the switch sits outside the row loop.
template <int TW>
__device__ __forceinline__ void frame_dh_rows(Frame &T, const JointRec &J, const JointVal &v) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float c0 = T.r[3 * i], c1 = T.r[3 * i + 1], c2 = T.r[3 * i + 2];
        const float n0 = fmaf(v.c, c0, v.s * c1);
        const float n1 = fmaf(v.c, c1, -v.s * c0);
        T.p[i] = fmaf(J.a, n0, fmaf(v.d, c2, T.p[i]));
        T.r[3 * i] = n0;
        if (TW == kTwist0) {
            T.r[3 * i + 1] = n1;
        } else if (TW == kTwistP90) {
            T.r[3 * i + 1] = c2;
            T.r[3 * i + 2] = -n1;
        } else if (TW == kTwistM90) {
            T.r[3 * i + 1] = -c2;
            T.r[3 * i + 2] = n1;
        } else {
            T.r[3 * i + 1] = fmaf(J.ca, n1, J.sa * c2);
            T.r[3 * i + 2] = fmaf(J.ca, c2, -J.sa * n1);
        }
    }
}

__device__ __forceinline__ void frame_dh_val(Frame &T, const JointRec &J, const JointVal &v) {
    switch (J.twist) {
    case kTwist0: frame_dh_rows<kTwist0>(T, J, v); break;
    case kTwistP90: frame_dh_rows<kTwistP90>(T, J, v); break;
    case kTwistM90: frame_dh_rows<kTwistM90>(T, J, v); break;
    default: frame_dh_rows<kTwistGeneral>(T, J, v); break;
    }
}

__device__ __forceinline__ void frame_dh(Frame &T, const JointRec &J, float q) {
    frame_dh_val(T, J, joint_val(J, q));
}

// Full joint update: optional mount, then the DH transform.
__device__ __forceinline__ void frame_joint_val(Frame &T, const JointRec &J, const JointVal &v) {
    if (J.has_mount) frame_mount(T, J.m);
    frame_dh_val(T, J, v);
}

__device__ __forceinline__ void frame_joint(Frame &T, const JointRec &J, float q) {
    frame_joint_val(T, J, joint_val(J, q));
}

// World position of a point given in the frame's coordinates.
__device__ __forceinline__ void frame_point(const Frame &T, float x, float y, float z, float &ox,
                                            float &oy, float &oz) {
    ox = fmaf(T.r[0], x, fmaf(T.r[1], y, fmaf(T.r[2], z, T.p[0])));
    oy = fmaf(T.r[3], x, fmaf(T.r[4], y, fmaf(T.r[5], z, T.p[1])));
    oz = fmaf(T.r[6], x, fmaf(T.r[7], y, fmaf(T.r[8], z, T.p[2])));
}

__device__ __forceinline__ void frame_rotate(const Frame &T, float x, float y, float z, float &ox,
                                             float &oy, float &oz) {
    ox = fmaf(T.r[0], x, fmaf(T.r[1], y, T.r[2] * z));
    oy = fmaf(T.r[3], x, fmaf(T.r[4], y, T.r[5] * z));
    oz = fmaf(T.r[6], x, fmaf(T.r[7], y, T.r[8] * z));
}

// Squared distance between the segments p1 + s d1 and p2 + t d2 (s, t in [0, 1]), given
// a = d1.d1 and e = d2.d2 with their reciprocals ia, ie (0 for a segment of zero length).  This
// is the closest-point construction for two segments (Ericson, Real-Time Collision Detection,
// sec. 5.1.9), without branches: s minimises the distance between the lines (0 when they are
// parallel), t is the closest parameter on the second segment for it, and when t leaves [0, 1]
// (or the second segment is a point) t is clamped and s recomputed for the clamped t.  The two
// points are always on the segments, so the result can only exceed the exact minimum through
// rounding in s and t.
__device__ __forceinline__ float seg_seg2(float p1x, float p1y, float p1z, float d1x, float d1y,
                                          float d1z, float a, float ia, float p2x, float p2y,
                                          float p2z, float d2x, float d2y, float d2z, float e,
                                          float ie) {
    const float rx = p1x - p2x, ry = p1y - p2y, rz = p1z - p2z;
    const float b = fmaf(d1x, d2x, fmaf(d1y, d2y, d1z * d2z));
    const float c = fmaf(d1x, rx, fmaf(d1y, ry, d1z * rz));
    const float f = fmaf(d2x, rx, fmaf(d2y, ry, d2z * rz));
    const float den = fmaf(a, e, -b * b);
    float s = den > 1e-6f * a * e
                  ? fminf(fmaxf(fmaf(b, f, -c * e) * __builtin_amdgcn_rcpf(den), 0.0f), 1.0f)
                  : 0.0f;
    const float t = fmaf(b, s, f) * ie;
    const float tc = fminf(fmaxf(t, 0.0f), 1.0f);
    if (t != tc || e == 0.0f) s = fminf(fmaxf(fmaf(tc, b, -c) * ia, 0.0f), 1.0f);
    const float x = fmaf(-tc, d2x, fmaf(s, d1x, rx));
    const float y = fmaf(-tc, d2y, fmaf(s, d1y, ry));
    const float z = fmaf(-tc, d2z, fmaf(s, d1z, rz));
    return fmaf(x, x, fmaf(y, y, z * z));
}

// ---------------------------------------------------------------------------------------
// Overlap tests of a robot sphere (centre c, radius r > 0) with one primitive.  Collision
// means clearance sd(c) - r < 0; each test is that inequality rewritten without a square
// root where possible (sd >= 0 outside, and any centre inside a convex primitive overlaps).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ bool hit_sphere(float cx, float cy, float cz, float r, float4 s) {
    const float dx = cx - s.x, dy = cy - s.y, dz = cz - s.z;
    const float rr = r + s.w;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rr * rr;
}

// Capsule (A = p0, radius; B = u, 1/|u|^2): distance to the clamped closest segment point.
__device__ __forceinline__ bool hit_capsule(float cx, float cy, float cz, float r, float4 A,
                                            float4 B) {
    const float wx = cx - A.x, wy = cy - A.y, wz = cz - A.z;
    float t = fmaf(wx, B.x, fmaf(wy, B.y, wz * B.z)) * B.w;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const float dx = fmaf(-t, B.x, wx), dy = fmaf(-t, B.y, wy), dz = fmaf(-t, B.z, wz);
    const float rr = r + A.w;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rr * rr;
}

// Flat-capped cylinder (A = centre, half height; B = unit axis, radius).
__device__ __forceinline__ bool hit_cylinder(float cx, float cy, float cz, float r, float4 A,
                                             float4 B) {
    const float vx = cx - A.x, vy = cy - A.y, vz = cz - A.z;
    const float h = fmaf(vx, B.x, fmaf(vy, B.y, vz * B.z));
    const float rx = fmaf(-h, B.x, vx), ry = fmaf(-h, B.y, vy), rz = fmaf(-h, B.z, vz);
    const float rho = sqrtf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
    const float x = fmaxf(rho - B.w, 0.0f);
    const float y = fmaxf(fabsf(h) - A.w, 0.0f);
    return fmaf(x, x, y * y) < r * r;
}

// Oriented box (three rows (column k of R, e_k) and the centre).
__device__ __forceinline__ bool hit_box(float cx, float cy, float cz, float r, float4 X,
                                        float4 Y, float4 Z, float4 O) {
    const float vx = cx - O.x, vy = cy - O.y, vz = cz - O.z;
    const float qx = fmaxf(fabsf(fmaf(X.x, vx, fmaf(X.y, vy, X.z * vz))) - X.w, 0.0f);
    const float qy = fmaxf(fabsf(fmaf(Y.x, vx, fmaf(Y.y, vy, Y.z * vz))) - Y.w, 0.0f);
    const float qz = fmaxf(fabsf(fmaf(Z.x, vx, fmaf(Z.y, vy, Z.z * vz))) - Z.w, 0.0f);
    return fmaf(qx, qx, fmaf(qy, qy, qz * qz)) < r * r;
}

// ---------------------------------------------------------------------------------------
// Signed distance and its gradient (unit direction of steepest increase), for the cost.
// Kinks follow fixed conventions: zero direction at a sphere centre or on a capsule axis;
// inside a box the face of the largest q component (lowest axis on ties, sign(0) = +1);
// inside a cylinder the cap when it is no farther than the side.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float sd_grad_point(float cx, float cy, float cz, float fx, float fy,
                                               float fz, float &gx, float &gy, float &gz) {
    const float dx = cx - fx, dy = cy - fy, dz = cz - fz;
    const float n = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    const float inv = n > 0.0f ? 1.0f / n : 0.0f;
    gx = dx * inv;
    gy = dy * inv;
    gz = dz * inv;
    return n;
}

__device__ __forceinline__ float sd_sphere(float cx, float cy, float cz, float4 s, float &gx,
                                           float &gy, float &gz) {
    return sd_grad_point(cx, cy, cz, s.x, s.y, s.z, gx, gy, gz) - s.w;
}

__device__ __forceinline__ float sd_capsule(float cx, float cy, float cz, float4 A, float4 B,
                                            float &gx, float &gy, float &gz) {
    const float wx = cx - A.x, wy = cy - A.y, wz = cz - A.z;
    float t = fmaf(wx, B.x, fmaf(wy, B.y, wz * B.z)) * B.w;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    return sd_grad_point(cx, cy, cz, fmaf(t, B.x, A.x), fmaf(t, B.y, A.y), fmaf(t, B.z, A.z),
                         gx, gy, gz) - A.w;
}

__device__ __forceinline__ float sd_cylinder(float cx, float cy, float cz, float4 A, float4 B,
                                             float &gx, float &gy, float &gz) {
    const float vx = cx - A.x, vy = cy - A.y, vz = cz - A.z;
    const float h = fmaf(vx, B.x, fmaf(vy, B.y, vz * B.z));
    const float rx = fmaf(-h, B.x, vx), ry = fmaf(-h, B.y, vy), rz = fmaf(-h, B.z, vz);
    const float rho = sqrtf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
    const float inv = rho > 0.0f ? 1.0f / rho : 0.0f;
    const float ux = rx * inv, uy = ry * inv, uz = rz * inv;
    const float ah = fabsf(h), sh = h >= 0.0f ? 1.0f : -1.0f;
    if (ah <= A.w && rho <= B.w) {
        const float a = A.w - ah, b = B.w - rho;
        if (a <= b) {
            gx = sh * B.x; gy = sh * B.y; gz = sh * B.z;
        } else {
            gx = ux; gy = uy; gz = uz;
        }
        return -fminf(a, b);
    }
    const float x = fmaxf(rho - B.w, 0.0f), y = fmaxf(ah - A.w, 0.0f);
    const float n = sqrtf(fmaf(x, x, y * y));
    const float in = 1.0f / n;
    gx = (x * ux + y * sh * B.x) * in;
    gy = (x * uy + y * sh * B.y) * in;
    gz = (x * uz + y * sh * B.z) * in;
    return n;
}

__device__ __forceinline__ float sd_box(float cx, float cy, float cz, float4 X, float4 Y,
                                        float4 Z, float4 O, float &gx, float &gy, float &gz) {
    const float vx = cx - O.x, vy = cy - O.y, vz = cz - O.z;
    const float p0 = fmaf(X.x, vx, fmaf(X.y, vy, X.z * vz));
    const float p1 = fmaf(Y.x, vx, fmaf(Y.y, vy, Y.z * vz));
    const float p2 = fmaf(Z.x, vx, fmaf(Z.y, vy, Z.z * vz));
    const float q0 = fabsf(p0) - X.w, q1 = fabsf(p1) - Y.w, q2 = fabsf(p2) - Z.w;
    const float m0 = fmaxf(q0, 0.0f), m1 = fmaxf(q1, 0.0f), m2 = fmaxf(q2, 0.0f);
    const float o2 = fmaf(m0, m0, fmaf(m1, m1, m2 * m2));
    const float s0 = p0 >= 0.0f ? 1.0f : -1.0f, s1 = p1 >= 0.0f ? 1.0f : -1.0f,
                s2 = p2 >= 0.0f ? 1.0f : -1.0f;
    float l0, l1, l2, sd;
    if (o2 > 0.0f) {
        const float n = sqrtf(o2);
        const float in = 1.0f / n;
        l0 = s0 * m0 * in;
        l1 = s1 * m1 * in;
        l2 = s2 * m2 * in;
        sd = n;
    } else {
        const int k = (q1 > q0) ? ((q2 > q1) ? 2 : 1) : ((q2 > q0) ? 2 : 0);
        l0 = k == 0 ? s0 : 0.0f;
        l1 = k == 1 ? s1 : 0.0f;
        l2 = k == 2 ? s2 : 0.0f;
        sd = fmaxf(q0, fmaxf(q1, q2));
    }
    // back to world: R * l, with R's columns stored as X, Y, Z
    gx = fmaf(X.x, l0, fmaf(Y.x, l1, Z.x * l2));
    gy = fmaf(X.y, l0, fmaf(Y.y, l1, Z.y * l2));
    gz = fmaf(X.z, l0, fmaf(Y.z, l1, Z.z * l2));
    return sd;
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

}  // namespace vk
