// Device helpers shared by the gfx950 kernels of libcvw: cross-lane moves inside
// 16-lane DPP rows, physical fluxes and interface fluxes.
#pragma once

#include <hip/hip_runtime.h>

#include "cvw_internal.h"

namespace cvw {

// ---------------------------------------------------------------------------
// DPP cross-lane moves.  A cell of a tensor-product element occupies one DPP
// row of 16 lanes, node (a, b) on lane a + 4 b of the row.
// ---------------------------------------------------------------------------
// Every pattern used here (quad_perm, row_ror) reads a lane of the same row,
// so no source is out of range: the moves need no old value and can be folded
// into the consuming VOP2 instruction by the compiler.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dppd(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = dppi<CTRL>(static_cast<int>(v & 0xffffffffLL));
  const int hi = dppi<CTRL>(static_cast<int>(v >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// value of lane i of the own quad (= node (i, b) of the own row b)
template <int I>
__device__ __forceinline__ float qbcast(float x) {
  return dpp<(I | (I << 2) | (I << 4) | (I << 6))>(x);
}
// rotation by 4 S lanes inside the 16-lane row: a value of the same column a
// from another row; which row it came from is tracked by rotating the row index
template <int S>
__device__ __forceinline__ float rrot(float x) {
  if constexpr (S == 0) return x; else return dpp<(0x120 | (4 * S))>(x);
}
template <int S>
__device__ __forceinline__ int rroti(int x) {
  if constexpr (S == 0) return x; else return dppi<(0x120 | (4 * S))>(x);
}

// value of lane N of the own 16-lane row (row_newbcast, gfx90a and later)
template <int N>
__device__ __forceinline__ double rowbcastd(double x) {
  return dppd<(0x150 | N)>(x);
}
// sum over the four lanes of the own quad (every lane receives bitwise the
// same value: butterfly order, no contraction, as for row_sum)
__device__ __forceinline__ float quad_sum(float x) {
#pragma clang fp contract(off)
  x = x + dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  return x;
}

__device__ __forceinline__ double quad_sumd(double x) {
#pragma clang fp contract(off)
  x = x + dppd<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dppd<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  return x;
}

template <int I>
__device__ __forceinline__ double qbcastd(double x) {
  return dppd<(I | (I << 2) | (I << 4) | (I << 6))>(x);
}
template <int S>
__device__ __forceinline__ double rrotd(double x) {
  if constexpr (S == 0) return x; else return dppd<(0x120 | (4 * S))>(x);
}

// Cross-lane dot products with the DPP source fused into the multiply-add
// (v_fmac_f32 with DPP; the compiler does not fuse DPP moves into
// multiply-adds, so each term would otherwise cost a move and an FMA).  The
// leading s_nop gives the two wait states a DPP read of a VGPR written by the
// previous VALU instruction needs; the other reads in a block are of the same
// source.  All sources lie inside the own 16-lane row.
#define CVW_DPP_TAIL " row_mask:0xf bank_mask:0xf bound_ctrl:1"
// sum_i c[i] x(lane i of the own quad)
__device__ __forceinline__ float qdot4(float x, const float (&c)[4]) {
  float a;
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,1,1]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %4 quad_perm:[2,2,2,2]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %5 quad_perm:[3,3,3,3]" CVW_DPP_TAIL
      : "=&v"(a) : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
  return a;
}
// a = sum_i c[i] x(lane i of the quad), b = sum_i d[i] x(lane i of the quad)
__device__ __forceinline__ void qdot4x2(float x, const float (&c)[4], const float (&d)[4], float& a, float& b) {
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %2, %3 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_mul_f32_dpp %1, %2, %7 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %2, %4 quad_perm:[1,1,1,1]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %8 quad_perm:[1,1,1,1]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %2, %5 quad_perm:[2,2,2,2]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %9 quad_perm:[2,2,2,2]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %2, %6 quad_perm:[3,3,3,3]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %10 quad_perm:[3,3,3,3]" CVW_DPP_TAIL
      : "=&v"(a), "=&v"(b)
      : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(d[0]), "v"(d[1]), "v"(d[2]), "v"(d[3]));
}
// Degree-1 packed cells (node (a, b) on lane a + 2 b of a quad): the pair
// along x, c0 x(0, b) + c1 x(1, b), and the pair along y, c0 x(a, 0) + c1 x(a, 1).
__device__ __forceinline__ float qx2(float x, float c0, float c1) {
  float r;
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %1, %2 quad_perm:[0,0,2,2]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,3,3]" CVW_DPP_TAIL
      : "=&v"(r) : "v"(x), "v"(c0), "v"(c1));
  return r;
}
__device__ __forceinline__ float qy2(float x, float c0, float c1) {
  float r;
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %1, %2 quad_perm:[0,1,0,1]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[2,3,2,3]" CVW_DPP_TAIL
      : "=&v"(r) : "v"(x), "v"(c0), "v"(c1));
  return r;
}
__device__ __forceinline__ float quad_max(float x) {
  x = fmaxf(x, dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x));
  x = fmaxf(x, dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x));
  return x;
}

// r + c0 x(lane 0 of the quad) + c3 x(lane 3 of the quad)
__device__ __forceinline__ float qfma03(float r, float x, float c0, float c3) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[3,3,3,3]" CVW_DPP_TAIL
      : "+v"(r) : "v"(x), "v"(c0), "v"(c3));
  return r;
}
// c[0] x + sum_{s=1..3} c[s] x(lane rotated by 4 s in the row)  (rows (b - s) & 3)
__device__ __forceinline__ float rdot4(float x, const float (&c)[4]) {
  float a;
  asm("v_mul_f32 %0, %1, %2\n\t"
      "s_nop 0\n\t"
      "v_fmac_f32_dpp %0, %1, %3 row_ror:4" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %4 row_ror:8" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %5 row_ror:12" CVW_DPP_TAIL
      : "=&v"(a) : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
  return a;
}
__device__ __forceinline__ void rdot4x2(float x, const float (&c)[4], const float (&d)[4], float& a, float& b) {
  asm("v_mul_f32 %0, %2, %3\n\t"
      "v_mul_f32 %1, %2, %7\n\t"
      "v_fmac_f32_dpp %0, %2, %4 row_ror:4" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %8 row_ror:4" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %2, %5 row_ror:8" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %9 row_ror:8" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %2, %6 row_ror:12" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %1, %2, %10 row_ror:12" CVW_DPP_TAIL
      : "=&v"(a), "=&v"(b)
      : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(d[0]), "v"(d[1]), "v"(d[2]), "v"(d[3]));
}

// Degree-1 and degree-2 variants over the lanes / rows that hold nodes:
// quad lanes 0..p; for p = 1 the rows 0, 1 are reached by the rotations 4
// and 12 (rotation 8 brings only unused rows).
__device__ __forceinline__ float qdot2(float x, const float (&c)[4]) {
  float a;
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,1,1]" CVW_DPP_TAIL
      : "=&v"(a) : "v"(x), "v"(c[0]), "v"(c[1]));
  return a;
}
__device__ __forceinline__ float qdot3(float x, const float (&c)[4]) {
  float a;
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,1,1]" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %4 quad_perm:[2,2,2,2]" CVW_DPP_TAIL
      : "=&v"(a) : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]));
  return a;
}
__device__ __forceinline__ float rdot3p1(float x, const float (&c)[4]) {
  float a;
  asm("v_mul_f32 %0, %1, %2\n\t"
      "s_nop 0\n\t"
      "v_fmac_f32_dpp %0, %1, %3 row_ror:4" CVW_DPP_TAIL "\n\t"
      "v_fmac_f32_dpp %0, %1, %4 row_ror:12" CVW_DPP_TAIL
      : "=&v"(a) : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[3]));
  return a;
}
// sum over the node lanes of the quad (p + 1 of them)
template <int P>
__device__ __forceinline__ float qdotp(float x, const float (&c)[4]) {
  if constexpr (P == 1) return qdot2(x, c);
  else if constexpr (P == 2) return qdot3(x, c);
  else return qdot4(x, c);
}
// sum over the node rows of the column
template <int P>
__device__ __forceinline__ float rdotp(float x, const float (&c)[4]) {
  if constexpr (P == 1) return rdot3p1(x, c);
  else return rdot4(x, c);
}

// Raw buffer access (gfx9 resource word 3 = 0x00020000: 32-bit data format):
// a uniform base in scalar registers, a 32-bit per-lane byte offset and a
// uniform 32-bit byte offset, no 64-bit address arithmetic per lane.  Offsets
// at or beyond `bytes` read 0 and drop stores (range-checked by the hardware).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(voff),
                                                                        static_cast<int>(soff), 0));
}
__device__ __forceinline__ void buf_store(float x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, static_cast<int>(voff),
                                        static_cast<int>(soff), 0);
}

// Sums / maxima over the 16 lanes of a row.  Butterfly order (lane i pairs
// with i^1, i^2, then the mirrored lane of the other quad and of the other half
// row): every lane adds the same two partial values, so all 16 lanes receive
// bitwise the same result.  Contraction is off so that a product feeding the
// sum is not fused into its first addition on one side of a pair only.
__device__ __forceinline__ float row_sum(float x) {
#pragma clang fp contract(off)
  x = x + dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  x = x + dpp<0x141>(x);
  x = x + dpp<0x140>(x);
  return x;
}
__device__ __forceinline__ double row_sumd(double x) {
#pragma clang fp contract(off)
  x = x + dppd<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dppd<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  x = x + dppd<0x141>(x);
  x = x + dppd<0x140>(x);
  return x;
}
__device__ __forceinline__ float row_max(float x) {
  x = fmaxf(x, dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x));
  x = fmaxf(x, dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x));
  x = fmaxf(x, dpp<0x141>(x));
  x = fmaxf(x, dpp<0x140>(x));
  return x;
}

// ---------------------------------------------------------------------------
// Fluxes (single precision).  fp = flux parameters, lam_g = global wave-speed
// bound (0 = local).
// ---------------------------------------------------------------------------
// hardware reciprocal (1 ulp): the hot kernels divide through it
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// hardware square root (v_sqrt_f32, about 1 ulp): the correctly rounded
// sqrtf costs a dozen instructions of range scaling and correction
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// sin and cos together (the KPP flux): the hardware v_sin_f32 / v_cos_f32,
// whose argument is in revolutions (valid within +-256 revolutions); the
// scaling by 1/(2 pi) rounds the argument by 6e-8 relative, about 1e-6
// absolute at |x| = 16.  Beyond |x| = 1000 the library functions.
__device__ __forceinline__ void kpp_sincos(float x, float& s, float& c) {
  if (fabsf(x) > 1.0e3f) {
    s = sinf(x);
    c = cosf(x);
    return;
  }
  const float rev = x * 0.159154943f;
  s = __builtin_amdgcn_sinf(rev);
  c = __builtin_amdgcn_cosf(rev);
}

template <int FLUX> struct NVar { static constexpr int value = 1; };
template <> struct NVar<CVW_EULER> { static constexpr int value = 4; };

template <int FLUX>
__device__ __forceinline__ void phys_flux(const MethodScalars& ms, const float* u, float x, float y,
                                          float* fx, float* fy) {
  if constexpr (FLUX == CVW_ADVECT_CONST) {
    fx[0] = ms.fp[0] * u[0];
    fy[0] = ms.fp[1] * u[0];
  } else if constexpr (FLUX == CVW_ADVECT_ROT) {
    const float vx = ms.fp[2] * (ms.fp[1] - y), vy = ms.fp[2] * (x - ms.fp[0]);
    fx[0] = vx * u[0];
    fy[0] = vy * u[0];
  } else if constexpr (FLUX == CVW_BURGERS) {
    const float h = 0.5f * u[0] * u[0];
    fx[0] = ms.fp[0] * h;
    fy[0] = ms.fp[1] * h;
  } else if constexpr (FLUX == CVW_KPP) {
    kpp_sincos(u[0], fx[0], fy[0]);
  } else {
    const float g = ms.fp[0];
    const float rho = u[0], inv = frcp(rho);
    const float vx = u[1] * inv, vy = u[2] * inv;
    const float p = (g - 1.0f) * (u[3] - 0.5f * rho * (vx * vx + vy * vy));
    fx[0] = u[1];
    fx[1] = u[1] * vx + p;
    fx[2] = u[2] * vx;
    fx[3] = (u[3] + p) * vx;
    fy[0] = u[2];
    fy[1] = u[1] * vy;
    fy[2] = u[2] * vy + p;
    fy[3] = (u[3] + p) * vy;
  }
}

// local maximum wave speed |f'(u)| (systems: |v| + c)
template <int FLUX>
__device__ __forceinline__ float wave_speed(const MethodScalars& ms, const float* u, float x, float y) {
  if constexpr (FLUX == CVW_ADVECT_CONST) {
    return fsqrt(ms.fp[0] * ms.fp[0] + ms.fp[1] * ms.fp[1]);
  } else if constexpr (FLUX == CVW_ADVECT_ROT) {
    const float vx = ms.fp[2] * (ms.fp[1] - y), vy = ms.fp[2] * (x - ms.fp[0]);
    return fsqrt(vx * vx + vy * vy);
  } else if constexpr (FLUX == CVW_BURGERS) {
    return fabsf(u[0]) * fsqrt(ms.fp[0] * ms.fp[0] + ms.fp[1] * ms.fp[1]);
  } else if constexpr (FLUX == CVW_KPP) {
    return 1.0f;
  } else {
    const float g = ms.fp[0];
    const float rho = u[0], inv = frcp(rho);
    const float vx = u[1] * inv, vy = u[2] * inv;
    const float p = (g - 1.0f) * (u[3] - 0.5f * rho * (vx * vx + vy * vy));
    return fsqrt(vx * vx + vy * vy) + fsqrt(fmaxf(g * p * inv, 0.0f));
  }
}

// interface flux f*(u-, u+, n): local Lax-Friedrichs for scalars, HLL with
// Exterior state at a boundary point of a 2D DG mesh: the neighbour table
// holds -(b + 1) for boundary face b, whose kind and state come with the
// method scalars.  Inflow imposes the state, a wall mirrors the normal
// momentum (Euler; a scalar law takes it as outflow), outflow copies the trace.
template <int FLUX>
__device__ __forceinline__ void ghost_state(const MethodScalars& ms, int32_t code, const float* um, float nx, float ny,
                                            float* up) {
  constexpr int NV = NVar<FLUX>::value;
  const int32_t b = -code - 1;
  const int kind = ms.bck[b];
#pragma unroll
  for (int v = 0; v < NV; ++v) up[v] = (kind == CVW_BC_INFLOW) ? ms.bcs[4 * b + v] : um[v];
  if constexpr (FLUX == CVW_EULER) {
    if (kind == CVW_BC_WALL) {
      const float mn = um[1] * nx + um[2] * ny;
      up[1] = fmaf(-2.0f * mn, nx, um[1]);
      up[2] = fmaf(-2.0f * mn, ny, um[2]);
    }
  }
}

// Davis wave-speed estimates for the Euler equations
template <int FLUX>
__device__ __forceinline__ void num_flux(const MethodScalars& ms, const float* um, const float* up, float nx,
                                         float ny, float x, float y, float* fs) {
  if constexpr (FLUX == CVW_EULER) {
    // velocities, pressure and sound speed once per state
    const float g = ms.fp[0];
    const float im = frcp(um[0]), ip = frcp(up[0]);
    const float vxm = um[1] * im, vym = um[2] * im, vxp = up[1] * ip, vyp = up[2] * ip;
    const float pm = (g - 1.0f) * (um[3] - 0.5f * um[0] * (vxm * vxm + vym * vym));
    const float pp = (g - 1.0f) * (up[3] - 0.5f * up[0] * (vxp * vxp + vyp * vyp));
    const float vm = vxm * nx + vym * ny, vp = vxp * nx + vyp * ny;
    const float cm = fsqrt(fmaxf(g * pm * im, 0.0f)), cp = fsqrt(fmaxf(g * pp * ip, 0.0f));
    const float SL = fminf(vm - cm, vp - cp);
    const float SR = fmaxf(vm + cm, vp + cp);
    // normal fluxes F.n of both states
    const float mnm = um[0] * vm, mnp = up[0] * vp;
    float Fm[4], Fp[4];
    Fm[0] = mnm;
    Fm[1] = um[1] * vm + pm * nx;
    Fm[2] = um[2] * vm + pm * ny;
    Fm[3] = (um[3] + pm) * vm;
    Fp[0] = mnp;
    Fp[1] = up[1] * vp + pp * nx;
    Fp[2] = up[2] * vp + pp * ny;
    Fp[3] = (up[3] + pp) * vp;
    const float inv = frcp(SR - SL);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float mid = (SR * Fm[v] - SL * Fp[v] + SL * SR * (up[v] - um[v])) * inv;
      fs[v] = (SL >= 0.0f) ? Fm[v] : ((SR <= 0.0f) ? Fp[v] : mid);
    }
  } else {
    float fxm[1], fym[1], fxp[1], fyp[1];
    phys_flux<FLUX>(ms, um, x, y, fxm, fym);
    phys_flux<FLUX>(ms, up, x, y, fxp, fyp);
    float lam;
    if (ms.lam_g > 0.0f) {
      lam = ms.lam_g;
    } else if constexpr (FLUX == CVW_ADVECT_CONST) {
      lam = fabsf(ms.fp[0] * nx + ms.fp[1] * ny);
    } else if constexpr (FLUX == CVW_ADVECT_ROT) {
      lam = fabsf(ms.fp[2] * ((ms.fp[1] - y) * nx + (x - ms.fp[0]) * ny));
    } else if constexpr (FLUX == CVW_BURGERS) {
      lam = fmaxf(fabsf(um[0]), fabsf(up[0])) * fabsf(ms.fp[0] * nx + ms.fp[1] * ny);
    } else {
      // |f'(u) . n| = |cos u nx - sin u ny| = |fy nx - fx ny|
      lam = fmaxf(fabsf(fym[0] * nx - fxm[0] * ny), fabsf(fyp[0] * nx - fxp[0] * ny));
    }
    const float Fm = fxm[0] * nx + fym[0] * ny;
    const float Fp = fxp[0] * nx + fyp[0] * ny;
    fs[0] = 0.5f * (Fm + Fp) - 0.5f * lam * (up[0] - um[0]);
  }
}

template <int FLUX>
__device__ __forceinline__ bool state_admissible(const MethodScalars& ms, const float* u) {
  if constexpr (FLUX == CVW_EULER) {
    const float inv = frcp(u[0]);
    const float p = (ms.fp[0] - 1.0f) * (u[3] - 0.5f * (u[1] * u[1] + u[2] * u[2]) * inv);
    return u[0] > 0.0f && p > 0.0f;
  } else {
    return true;
  }
}

// ---------------------------------------------------------------------------
// bilinear quadrilateral geometry (vertex 0 absolute, others relative to it)
// ---------------------------------------------------------------------------
struct Geo {
  float x0, y0;          // vertex 0 (absolute)
  float d[4][2];         // vertex v - vertex 0
  float h[2];            // d^2 x / dxi deta (constant for a bilinear map)
};

__device__ __forceinline__ Geo load_geo(const float* __restrict__ g, int64_t e) {
  Geo G;
  const float* p = g + e * 8;
  G.x0 = p[0];
  G.y0 = p[1];
  G.d[0][0] = 0.0f;
  G.d[0][1] = 0.0f;
  for (int v = 1; v < 4; ++v) {
    G.d[v][0] = p[2 * v];
    G.d[v][1] = p[2 * v + 1];
  }
  for (int c = 0; c < 2; ++c) G.h[c] = 0.25f * (G.d[0][c] - G.d[1][c] + G.d[2][c] - G.d[3][c]);
  return G;
}

// bilinear map at (xi, eta): position relative to vertex 0, Jacobian J[a][b] = dx_a / dxi_b
__device__ __forceinline__ void geo_eval(const Geo& G, float xi, float eta, float& px, float& py, float J[2][2]) {
  const float sxv[4] = {-1.f, 1.f, 1.f, -1.f}, syv[4] = {-1.f, -1.f, 1.f, 1.f};
  px = py = 0.0f;
  J[0][0] = J[0][1] = J[1][0] = J[1][1] = 0.0f;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float N = 0.25f * (1.0f + sxv[v] * xi) * (1.0f + syv[v] * eta);
    const float Nx = 0.25f * sxv[v] * (1.0f + syv[v] * eta);
    const float Ny = 0.25f * syv[v] * (1.0f + sxv[v] * xi);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      J[c][0] = fmaf(Nx, G.d[v][c], J[c][0]);
      J[c][1] = fmaf(Ny, G.d[v][c], J[c][1]);
    }
    px = fmaf(N, G.d[v][0], px);
    py = fmaf(N, G.d[v][1], py);
  }
}

// XCD-aware block order: consecutive logical blocks land on the same XCD so
// that a block's neighbours (one grid row away) are served by the same L2.
// bfloat16 bit patterns, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks_padded) {
  const int64_t per = nblocks_padded >> 3;
  return (bid & 7) * per + (bid >> 3);
}

}  // namespace cvw
