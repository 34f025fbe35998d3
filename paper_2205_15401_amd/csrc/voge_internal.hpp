// voge_internal.hpp -- records, constants and device helpers shared by the
// HIP sources of libvoge (gfx950 / CDNA4).  Not part of the public C ABI.
//
// Data layout in HBM (per item -- one kernel set seen by one camera --,
// written by the prep kernels; the items' slices are concatenated):
//   CullRec  cull[N]  16 B  screen bbox + depth-bucket floor, in depth order
//   TraceRec rec[N]   96 B  per-kernel ray-tracing coefficients, same order
//   GeoRec   geo[N]   80 B  camera-space centre and inverse covariance (backward)
// Within an item the order is ascending in the lower bound of the ray
// parameter of the kernel's eta-ellipsoid (bucketed), so a block of pixels
// can stop scanning once every pixel holds K kernels that are all nearer
// than the next record's floor.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace voge {

constexpr int TILE = 16;               // screen tile edge (pixels)
constexpr int TILE_THREADS = TILE * TILE;
constexpr int WAVE = 64;
constexpr int RANK_BITS = 24;          // low bits of a K-buffer key hold the kernel's rank
constexpr uint64_t RANK_MASK = (1ull << RANK_BITS) - 1;
constexpr int MAX_KERNELS = 1 << RANK_BITS;
constexpr int MAX_K = 64;
constexpr int MAX_IMAGE = 32767;       // bbox rows/cols are stored as int16
constexpr uint32_t KEY_CULLED = 0xFFFFFFFFu;

// device status bits (sticky, in the workspace header)
constexpr int ST_NOTSPD = 1;
constexpr int ST_NONFINITE = 2;

struct __align__(16) CullRec {
    int16_t i0, i1, j0, j1;   // inclusive pixel rows / columns that can see the kernel
    float tlo;                // lower bound of the ray parameter (D' units) of its peak
    uint32_t pad;
};

// Ray tracing of one kernel along D' = (u, v, F), u = i - O_y, v = j - O_x:
//   a(u,v) = D'^T S D' = u (A0 u + A1 v + A2) + v (A3 v + A4) + A5
//   b(u,v) = D'^T S M  = B0 u + B1 v + B2
//   l = b / a,  -2 q = M^T S M - b l = c - b l
struct __align__(16) TraceRec {
    double A0, A1, A2, A3, A4, A5;
    double B0, B1, B2;
    double c;
    float tlo;
    uint32_t idx;             // original kernel index
    uint32_t rank;            // position in depth-bound order
    uint32_t pad;
};
static_assert(sizeof(TraceRec) == 96, "TraceRec is 96 bytes");

struct __align__(8) GeoRec {
    double M[3];              // camera-space centre
    double S[6];              // camera-space inverse covariance xx, xy, xz, yy, yz, zz
    uint32_t idx;             // original kernel index
    uint32_t pad;
};
static_assert(sizeof(GeoRec) == 80, "GeoRec is 80 bytes");

struct CamDev {               // camera as passed to kernels
    float R[9], T[3];
    float F, cx, cy;
    int H, W;
};

struct WsHeader {             // first bytes of every workspace
    int status;               // sticky device status bits
    int pad[63];
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t float_order_key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// The same address as a pointer into the global address space: loads and
// stores through it are global accesses, not flat ones (a flat access also
// counts against the LDS / scalar-load wait counter, so waiting for it
// waits for those too).  For pointers read from memory, whose address space
// the compiler cannot infer.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
    return (gptr<T>)p;
}

// Whole-record loads and stores through global pointers (the records'
// implicit copy operators take generic references, which a global object
// cannot bind to): 16-byte vectors as one access, records member by member.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ld_f4(gptr<const float4> p) {
    const f32x4 v = *(gptr<const f32x4>)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void st_f4(gptr<float4> p, float4 a) {
    f32x4 v;
    v.x = a.x;
    v.y = a.y;
    v.z = a.z;
    v.w = a.w;
    *(gptr<f32x4>)p = v;
}

// Float atomic add to global memory (no return value).
__device__ __forceinline__ void global_add(float* p, float v) {
    __builtin_amdgcn_global_atomic_fadd_f32(gp(p), v);
}

// Wave votes over the active lanes, taken on the lane mask itself (no
// round trip of the predicate through a vector register).
__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Symmetric 3x3 inverse by cofactors, FP64.  Returns false unless the matrix
// is symmetric positive definite (checked by its Cholesky pivots) and finite.
__device__ __forceinline__ bool spd_inverse6(const double s[6], double inv[6]) {
    const double xx = s[0], xy = s[1], xz = s[2], yy = s[3], yz = s[4], zz = s[5];
    // Cholesky pivots: xx, yy - xy^2/xx, and the Schur complement of zz
    if (!(xx > 0.0)) return false;
    const double p1 = yy - xy * xy / xx;
    if (!(p1 > 0.0)) return false;
    const double l21 = yz - xy * xz / xx;
    const double p2 = zz - xz * xz / xx - l21 * l21 / p1;
    if (!(p2 > 0.0)) return false;
    const double c00 = yy * zz - yz * yz;
    const double c01 = xz * yz - xy * zz;
    const double c02 = xy * yz - xz * yy;
    const double c11 = xx * zz - xz * xz;
    const double c12 = xy * xz - xx * yz;
    const double c22 = xx * yy - xy * xy;
    const double det = xx * c00 + xy * c01 + xz * c02;
    if (!(det > 0.0) || !isfinite(det)) return false;
    const double r = 1.0 / det;
    inv[0] = c00 * r; inv[1] = c01 * r; inv[2] = c02 * r;
    inv[3] = c11 * r; inv[4] = c12 * r; inv[5] = c22 * r;
    return isfinite(inv[0]) && isfinite(inv[1]) && isfinite(inv[2]) &&
           isfinite(inv[3]) && isfinite(inv[4]) && isfinite(inv[5]);
}

// B = R A R^T for symmetric A (packed 6) and a row-major 3x3 R.
__device__ __forceinline__ void rotate_sym(const double R[9], const double A[6], double B[6]) {
    const double F[9] = {A[0], A[1], A[2], A[1], A[3], A[4], A[2], A[4], A[5]};
    double RA[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            RA[3 * r + c] = R[3 * r] * F[c] + R[3 * r + 1] * F[3 + c] + R[3 * r + 2] * F[6 + c];
    auto e = [&](int r, int c) { return RA[3 * r] * R[3 * c] + RA[3 * r + 1] * R[3 * c + 1] + RA[3 * r + 2] * R[3 * c + 2]; };
    B[0] = e(0, 0); B[1] = e(0, 1); B[2] = e(0, 2);
    B[3] = e(1, 1); B[4] = e(1, 2); B[5] = e(2, 2);
}

// The screen box of a cull record alone (its first 8 bytes).
struct CullBox {
    int16_t i0, i1, j0, j1;
};

__device__ __forceinline__ CullBox load_box(gptr<const CullRec> p) {
    CullBox c;
    c.i0 = p->i0;
    c.i1 = p->i1;
    c.j0 = p->j0;
    c.j1 = p->j1;
    return c;
}

__device__ __forceinline__ CullRec load_cull(gptr<const CullRec> p) {
    CullRec c;
    c.i0 = p->i0;
    c.i1 = p->i1;
    c.j0 = p->j0;
    c.j1 = p->j1;
    c.tlo = p->tlo;
    c.pad = 0;
    return c;
}

__device__ __forceinline__ GeoRec load_geo(gptr<const GeoRec> p) {
    GeoRec g;
#pragma unroll
    for (int i = 0; i < 3; ++i) g.M[i] = p->M[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) g.S[i] = p->S[i];
    g.idx = p->idx;
    g.pad = 0;
    return g;
}

}  // namespace voge
