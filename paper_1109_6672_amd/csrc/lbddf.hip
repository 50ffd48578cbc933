// lbddf.hip - gfx950 kernels and C ABI of the coupled double-distribution-
// function thermal lattice Boltzmann model on D2Q9 (Li, Luo, He, Gao & Tao).
//
// Design (MI355X / CDNA4):
//  * Structure-of-arrays populations, 18 planes (f^ then h-) per buffer, two
//    buffers (A/B).  Within each half (f, h) the rows of the 9 planes are
//    interleaved, [y][a][x]: the 9 rows of one grid row sit next to each
//    other, which keeps the addresses that the wavefronts in flight touch in a
//    compact window (measured: ~10% more HBM throughput than whole planes
//    one after the other).  A buffer holds the post-collision values of the
//    previous step at each node's own index; a step pull-gathers them (Eq. 45
//    read backwards), collides, and stores into the other buffer at the
//    node's own index, so every load and store of a wavefront touches 64
//    consecutive nodes of one population row.
//  * Deviation storage and arithmetic: a plane holds x - x_rest, where x_rest
//    is the equilibrium of the rest state (rho0, 0, T0).  Moments, equilibria,
//    the collision and the codec all work on these deviations, which keeps
//    FP32 (and the 16-bit codecs) accurate for the small perturbations of
//    low-Mach flows.
//  * A wavefront owns 64 aligned columns of a strip of R rows and marches
//    through it, one row per iteration; the wavefronts of a block own
//    adjacent tiles of one strip and march in lockstep (one barrier per row),
//    up on even strips and down on odd ones.  The x-neighbours of the
//    correction term's Q (Eq. 48-50) come from the adjacent lanes and, at the
//    tile edges, through LDS from the neighbouring wavefronts; the
//    y-neighbours come from the previous and the look-ahead row kept in
//    registers.  Only the two outer wavefronts of a block gather the columns
//    just outside it, for 32 rows at a time (one row per lane).  Each row is
//    gathered once, and neighbouring tiles and strips read the lines they
//    share at the same time, while those are in L2.
//  * Boundary nodes gather the populations of the interior node they
//    extrapolate from instead of their own (non-equilibrium extrapolation),
//    so the wavefront's loads stay uniform; the rebuild is a short divergent
//    branch on boundary lanes only.
//  * Work is swizzled over the 8 XCDs so that neighbouring strips, which
//    share halo rows and columns, run on the same L2.
//  * MFMA is not used: the step is a bandwidth-bound stencil, not a dense
//    contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "lbddf.h"

// Arithmetic type of the step: FP32, or FP64 in the library built with
// LB_ARITH_FP64 (liblbddf_fp64.so: same ABI and storage formats).
#ifdef LB_ARITH_FP64
typedef double real;
#else
typedef float real;
#endif

namespace {

constexpr int kWave = 64;
constexpr int kTile = 64;  // owned columns per wavefront (aligned)
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kHaloRows = kWave / 2;  // rows served by one halo gather (one per lane half)
// wavefronts per block of the single-grid step, marching in lockstep
// (measured best on 8192^2: 8 for FP32 storage, 4 for the 16-bit codecs)
template <int ST> constexpr int kLock = ST == LB_STORE_F32 ? 8 : 4;
constexpr int kRedBlocks = 1024;
constexpr int kNred = 8;
constexpr int kPlanePadBytes = 4096;  // appended to each plane's share of a half

enum : int { K_INTERIOR = 0, K_DIRICHLET = 1, K_ADIABATIC = 2, K_INLET = 3, K_OUTLET = 4 };

// Everything a kernel needs, passed by value.
struct KArgs {
    int nx, ny, pitch;
    int rs;  // population row stride (elements): 9 pitch, the interleaved rows of a half
    int tiles_x, n_strips, strip_rows;
    int per_x, per_y;
    long long plane_bytes;  // a half (f or h) spans 9 plane_bytes
    unsigned pstride;       // bytes from one population's row to the next one's
    int total, heat, corr, coupled, bgk, visc, rho_press, has_force;
    int dither;  // dithered FP32 sums in the bounded step (internal-energy grids)
    real rho0, E0, inv_E0, half_g, g, Pr;
    // relaxation for a constant tau_f
    real s_nu, s_e, s_z, s_q, s_rho, s_j, omega_h, kcoup;
    int tie_e, tie_z;
    // viscosity laws: mu3 = 3 mu_ref, r = cT theta = T / T_ref
    real mu3, cT, visc_n, sT;
    // sides x-, x+, y-, y+
    int side_kind[4];
    real side_ux[4], side_uy[4], side_dth[4];
    // inlet source (Eq. 53-54): amplitudes of u_x, rho - rho0 and theta - 1,
    // and 1 / period (steps); the phase comes from the time step on the device
    real in_u, in_rho, in_th;
    double in_rate;
    // time step of the state a launch reads (modulo 2^32)
    unsigned step;
};

// Reciprocal: hardware estimate plus one Newton step, so that rho * (j / rho)
// reproduces j without the systematic bias of the raw estimate.
// Model switches: Dyn reads them from the kernel arguments; Head fixes the
// ones of the main throughput configuration (total energy with the heating
// term, theta-coupled equilibria, correction term, no body force, MRT,
// constant tau_f) at compile time so that no dead branch is evaluated.
struct Dyn {
    static constexpr bool fixed = false, total = false, heat = false, coupled = false, corr = false,
                          force = false, bgk = false, ctau = false, precise = false;
};
// Dyn for grids with walls: FP64 moments and wall rebuild with FP32 storage
// (see MomType)
struct DynW : Dyn {
    static constexpr bool precise = true;
};
// Grids with walls in the cavity configuration (Sec. IV-C: internal energy,
// no heating term, coupled, correction term, gravity, MRT, a viscosity law
// other than constant tau) with compile-time switches: the dead paths of the
// runtime switches go, which takes the FP32 kernel from 236 VGPRs to 207 and
// the 16-bit one from 143 to 124 (four wavefronts per SIMD)
struct CavW {
    static constexpr bool fixed = true, total = false, heat = false, coupled = true, corr = true, force = true,
                          bgk = false, ctau = false, precise = true;
};
struct Head {
    static constexpr bool fixed = true, total = true, heat = true, coupled = true, corr = true, force = false,
                          bgk = false, ctau = true, precise = false;
};
#define F_TOTAL (F::fixed ? F::total : (bool)a.total)
#define F_HEAT (F::fixed ? F::heat : (bool)a.heat)
#define F_COUPLED (F::fixed ? F::coupled : (bool)a.coupled)
#define F_CORR (F::fixed ? F::corr : (bool)a.corr)
#define F_FORCE (F::fixed ? F::force : (bool)a.has_force)
#define F_BGK (F::fixed ? F::bgk : (bool)a.bgk)
#define F_CTAU (F::fixed ? F::ctau : (a.visc == LB_VISC_CONST_TAU))

__device__ __forceinline__ float frcp(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.f), r);
}
#ifdef LB_ARITH_FP64
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
#else
// FP64 reciprocal for the FP64 moments of the bounded-grid step: hardware
// estimate plus two Newton steps
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
#endif

// sin(pi x) in the arithmetic type
#ifndef LB_ARITH_FP64
__device__ __forceinline__ real sin_pi(real x) { return sinpif(x); }
#else
__device__ __forceinline__ real sin_pi(real x) { return sinpi(x); }
#endif

// readlane of a real (two 32-bit halves in FP64)
#ifndef LB_ARITH_FP64
__device__ __forceinline__ real readlane_real(real v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
#else
__device__ __forceinline__ real readlane_real(real v, int lane) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
    return __builtin_bit_cast(real, ((unsigned long long)hi << 32) | lo);
}
#endif

// ------------------------------------------------------------------ storage
// A population buffer is addressed through two raw buffer resources, one for
// the 9 f-planes and one for the 9 h-planes (each spans less than 4 GiB): the
// per-lane byte offset of the node goes in a VGPR, the plane offset in an
// SGPR, so no load or store spends vector instructions on 64-bit addresses.
typedef __amdgpu_buffer_rsrc_t Rsrc;
// cache policy of the population stores: non-temporal (each value is written
// once per step and read back only in the next step).  Loads stay cached:
// neighbouring lanes, tiles and the halo gather share their cache lines.
constexpr int kNT = 2;

struct Planes {
    Rsrc f, h;
    unsigned pb;  // bytes from one population's row to the next one's
};

__device__ __forceinline__ Planes planes(const char *base, const KArgs &a) {
    Planes P;
    const unsigned half = (unsigned)(9 * a.plane_bytes);
    P.f = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)half, 0x00020000);
    P.h = __builtin_amdgcn_make_buffer_rsrc((void *)(base + 9 * a.plane_bytes), (short)0, (int)half, 0x00020000);
    P.pb = a.pstride;
    return P;
}

typedef _Float16 H2 __attribute__((ext_vector_type(2)));
typedef __bf16 B2 __attribute__((ext_vector_type(2)));

// q is the plane (0..17); after unrolling it is a compile-time constant.
template <int ST> struct Codec;
template <> struct Codec<LB_STORE_F32> {
    static constexpr unsigned bytes = 4;
    static __device__ __forceinline__ real ld(const Planes &P, unsigned vo, int q) {
        const Rsrc r = q < 9 ? P.f : P.h;
        return (real)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, (q % 9) * P.pb, 0));
    }
    static __device__ __forceinline__ void st(const Planes &P, unsigned vo, real v, int q, unsigned rb) {
        const Rsrc r = q < 9 ? P.f : P.h;
#ifdef LB_ARITH_FP64
        // The FP64 value rounds stochastically to FP32: one step past the
        // round-to-nearest value f, towards v, with probability
        // |v - f| / (that step), so that the storage adds no systematic
        // drift to long runs (the random bits are the 24 high ones of rb)
        float f = (float)v;
        const real e = v - (real)f;
        if (e != real(0.) && f != 0.f) {
            const unsigned fb = __float_as_uint(f);
            const float g = __uint_as_float(((e > real(0.)) == (f > 0.f)) ? fb + 1u : fb - 1u);
            const real step = fabs((real)g - (real)f);
            if (fabs(e) > (real)(rb >> 8) * real(1. / 16777216.) * step) f = g;
        }
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(f), r, vo, (q % 9) * P.pb, kNT);
#else
        (void)rb;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)v), r, vo, (q % 9) * P.pb, kNT);
#endif
    }
};
// FP16 keeps deviation * 2^(8 + k_a), k_a = 1, 3, 5 for the rest, axis and
// diagonal velocities (about 1 / w_a): every plane then spans the same
// range, far above the FP16 subnormals and far below its maximum.  Powers of
// two make the scaling exact.
__device__ __forceinline__ real f16_scale(int q) {
    const int a = q % 9;
    return a == 0 ? real(512.) : (a < 5 ? real(2048.) : real(8192.));
}
template <> struct Codec<LB_STORE_F16> {
    static constexpr unsigned bytes = 2;
    static __device__ __forceinline__ real ld(const Planes &P, unsigned vo, int q) {
        const Rsrc r = q < 9 ? P.f : P.h;
        const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, vo, (q % 9) * P.pb, 0);
        // an FMA with a zero addend, not a product: it becomes one mixed-
        // precision FMA that converts and scales (a product of a converted
        // value stays two instructions when it has several users)
        return fma((real)__builtin_bit_cast(_Float16, b), real(1.) / f16_scale(q), real(0.));
    }
    // rb: random bits; the conversion rounds stochastically (gfx950's
    // v_cvt_sr_f16_f32 adds the high bits of rb below the kept mantissa of the
    // magnitude, then truncates), which leaves no systematic rounding bias in
    // steady flows.
    static __device__ __forceinline__ void st(const Planes &P, unsigned vo, real v, int q, unsigned rb) {
        const Rsrc r = q < 9 ? P.f : P.h;
        // the conversion writes one half of a register; the other half is
        // never stored, so the input's own register serves as the old value
        const float sv = (float)(v * f16_scale(q));
        const H2 h = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(H2, sv), sv, rb, false);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[0]), r, vo, (q % 9) * P.pb, kNT);
    }
};
template <> struct Codec<LB_STORE_BF16> {
    static constexpr unsigned bytes = 2;
    static __device__ __forceinline__ real ld(const Planes &P, unsigned vo, int q) {
        const Rsrc r = q < 9 ? P.f : P.h;
        const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, vo, (q % 9) * P.pb, 0);
        return __uint_as_float(((unsigned)b) << 16);
    }
    // stochastic rounding of the 16 dropped mantissa bits (see the FP16 codec)
    static __device__ __forceinline__ void st(const Planes &P, unsigned vo, real v, int q, unsigned rb) {
        const Rsrc r = q < 9 ? P.f : P.h;
        const B2 h = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(B2, (float)v), (float)v, rb, false);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[0]), r, vo, (q % 9) * P.pb, kNT);
    }
};

// --------------------------------------------------------- node primitives
// drho = rho - rho0, j = rho u (the momentum of Eq. 46 with the forcing note),
// u, dth = theta - 1; sf, sx, sy are the raw sums sum f, sum e f of the
// (possibly rebuilt) populations, which equal drho, jx and jy + rho g / 2 on
// interior nodes.
template <class T> struct MomT {
    T drho, rho, jx, jy, ux, uy, dth, sf, sx, sy;
};
typedef MomT<real> Mom;

// Type of the moments and of the moment-space non-equilibrium of a node.
// Bounded grids (walls, inlet, outlet) with FP32 storage compute them, and the
// rebuild of their boundary nodes, in FP64: there the populations deviate from
// the rest state by O(1) (large temperature differences, gravity
// stratification), and FP32 rounding of the sums and of the cancellation
// m - m_eq, repeated alike every step, biases the mass that the walls exchange
// and the flow over long runs.  On CDNA4 an FP64 FMA issues at the rate of a
// (non-packed) FP32 one; the cost is registers.  With 16-bit storage the
// rounding of the stored values dominates and FP32 suffices.
template <bool P> struct MomType { typedef real type; };
template <> struct MomType<true> { typedef double type; };
template <int ST, bool BC, class F> constexpr bool kPrecise = BC && F::precise && ST == LB_STORE_F32;

// Pull-gather (Eq. 45): population a of node (x, y) is the post-collision
// value stored at (x, y) - e_a, with periodic wrap.  Sources of a bounded
// axis are interior nodes, so their neighbours never leave the domain.
template <int ST>
__device__ __forceinline__ void gather(const KArgs &a, const Planes &S, int x, int y, real d[18]) {
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    xm += (xm < 0) ? a.nx : 0;
    xp -= (xp >= a.nx) ? a.nx : 0;
    ym += (ym < 0) ? a.ny : 0;
    yp -= (yp >= a.ny) ? a.ny : 0;
    const unsigned eb = Codec<ST>::bytes;
    const unsigned rm = (unsigned)ym * a.rs, rc = (unsigned)y * a.rs, rp = (unsigned)yp * a.rs;
    const unsigned o[9] = {(rc + x) * eb,  (rc + xm) * eb, (rm + x) * eb,  (rc + xp) * eb, (rp + x) * eb,
                           (rm + xm) * eb, (rm + xp) * eb, (rp + xp) * eb, (rp + xm) * eb};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        d[q] = Codec<ST>::ld(S, o[q], q);
        d[9 + q] = Codec<ST>::ld(S, o[q], 9 + q);
    }
}

// Eq. 46 with the forcing note (rho u = sum e f + a/2, a = (0, -rho g)) and
// Eq. 37 / the internal-energy form, written for deviations from rest.
template <class F, class T = real>
__device__ __forceinline__ MomT<T> moments(const KArgs &a, const real dr[18]) {
    MomT<T> m;
    T d[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) d[q] = (T)dr[q];
    const T s1 = (d[1] + d[3]) + (d[2] + d[4]);
    const T s2 = (d[5] + d[7]) + (d[6] + d[8]);
    m.drho = d[0] + (s1 + s2);
    const T jx = (d[1] - d[3]) + (d[5] - d[7]) + (d[8] - d[6]);
    const T jy = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
    m.sf = m.drho;
    m.sx = jx;
    m.sy = jy;
    m.rho = (T)a.rho0 + m.drho;
    const T ir = frcp(m.rho);
    m.jx = jx;
    m.jy = F_FORCE ? jy - (T)a.half_g * m.rho : jy;
    m.ux = m.jx * ir;
    m.uy = m.jy * ir;
    const T sh = ((d[9] + d[10]) + (d[11] + d[12])) + ((d[13] + d[14]) + (d[15] + d[16])) + d[17];
    const T e = (sh - m.drho * (T)a.E0) * ir;  // E - E0 (total) or (rho E_int - rho E0)/rho
    m.dth = F_TOTAL ? (e - T(0.5) * (m.ux * m.ux + m.uy * m.uy)) * (T)a.inv_E0 : e * (T)a.inv_E0;
    return m;
}

template <class T, class U> __device__ __forceinline__ MomT<T> mom_cast(const MomT<U> &u) {
    MomT<T> m;
    m.drho = (T)u.drho;
    m.rho = (T)u.rho;
    m.jx = (T)u.jx;
    m.jy = (T)u.jy;
    m.ux = (T)u.ux;
    m.uy = (T)u.uy;
    m.dth = (T)u.dth;
    m.sf = (T)u.sf;
    m.sx = (T)u.sx;
    m.sy = (T)u.sy;
    return m;
}

// Deviations of the equilibria Eq. 18a and Eq. 18b (or h = b R T f / 2) from
// the rest equilibria, lattice units (R T0 = 1/3), written with the momentum
// j = rho u so that the first moment of f_eq is j itself:
//   f_eq - f_rest = w [drho + c rho th - 1.5 j.u + (e.j)(B + 4.5 e.u)],
//   c = -1, 1/2, 2 and B = 3, 3 - 1.5 th, 3 + 3 th for |e|^2 = 0, 1, 2.
template <class F, class T>
__device__ __forceinline__ void equilibria(const KArgs &a, const MomT<T> &m, T fe[9], T he[9]) {
    const T w0 = T(4.) / T(9.), w1 = T(1.) / T(9.), w2 = T(1.) / T(36.);
    const T th = F_COUPLED ? m.dth : T(0.);  // theta_eq - 1
    const T ux = m.ux, uy = m.uy, jx = m.jx, jy = m.jy, drho = m.drho, rho = m.rho;
    const T ju = jx * ux + jy * uy;
    const T base = drho - T(1.5) * ju;
    const T rth = rho * th;
    const T A0 = base - rth, A1 = base + T(0.5) * rth, A2 = base + T(2.) * rth;
    const T B1 = T(3.) - T(1.5) * th, B2 = T(3.) + T(3.) * th;
    const T v5 = ux + uy, v6 = uy - ux, j5 = jx + jy, j6 = jy - jx;
    fe[0] = w0 * A0;
    fe[1] = w1 * (A1 + jx * (B1 + T(4.5) * ux));
    fe[3] = w1 * (A1 - jx * (B1 - T(4.5) * ux));
    fe[2] = w1 * (A1 + jy * (B1 + T(4.5) * uy));
    fe[4] = w1 * (A1 - jy * (B1 - T(4.5) * uy));
    fe[5] = w2 * (A2 + j5 * (B2 + T(4.5) * v5));
    fe[7] = w2 * (A2 - j5 * (B2 - T(4.5) * v5));
    fe[6] = w2 * (A2 + j6 * (B2 + T(4.5) * v6));
    fe[8] = w2 * (A2 - j6 * (B2 - T(4.5) * v6));
    const T u2 = ux * ux + uy * uy;
    if (F_TOTAL) {
        // h_eq - h_rest = w [rho0 (E - E0) + c (p theta - p0) + p (3 eu + 9 eu^2 - 3 u^2)] + E (f_eq - f_rest),
        // p (3 eu + 9 eu^2 - 3 u^2) = theta [(e.j)(1 + 3 e.u) - j.u] with p = rho theta / 3
        const T E = (T)a.E0 * (T(1.) + m.dth) + T(0.5) * u2;
        const T K0 = (T)a.rho0 * ((T)a.E0 * m.dth + T(0.5) * u2);
        const T third = T(1.) / T(3.);
        const T Pt = T(1.) + th;
        const T Pd = (drho + rth * (T(2.) + th)) * third;
        const T k0 = K0 - Pd - Pt * ju, k1 = K0 + T(0.5) * Pd - Pt * ju, k2 = K0 + T(2.) * Pd - Pt * ju;
        he[0] = w0 * k0 + E * fe[0];
        he[1] = w1 * (k1 + Pt * jx * (T(1.) + T(3.) * ux)) + E * fe[1];
        he[3] = w1 * (k1 - Pt * jx * (T(1.) - T(3.) * ux)) + E * fe[3];
        he[2] = w1 * (k1 + Pt * jy * (T(1.) + T(3.) * uy)) + E * fe[2];
        he[4] = w1 * (k1 - Pt * jy * (T(1.) - T(3.) * uy)) + E * fe[4];
        he[5] = w2 * (k2 + Pt * j5 * (T(1.) + T(3.) * v5)) + E * fe[5];
        he[7] = w2 * (k2 - Pt * j5 * (T(1.) - T(3.) * v5)) + E * fe[7];
        he[6] = w2 * (k2 + Pt * j6 * (T(1.) + T(3.) * v6)) + E * fe[6];
        he[8] = w2 * (k2 - Pt * j6 * (T(1.) - T(3.) * v6)) + E * fe[8];
    } else {
        const T c = (T)a.rho0 * (T)a.E0 * m.dth, Et = (T)a.E0 * (T(1.) + m.dth);
        he[0] = w0 * c + Et * fe[0];
#pragma unroll
        for (int q = 1; q < 5; ++q) he[q] = w1 * c + Et * fe[q];
#pragma unroll
        for (int q = 5; q < 9; ++q) he[q] = w2 * c + Et * fe[q];
    }
}

struct Relax {
    real s_nu, s_e, s_z, omega_h, kcoup;
};

// Per-node transport: tau_f = mu(T) / p + 1/2 (Sec. IV-C) for the viscosity
// laws, tau_h = (tau_f - 1/2)/Pr, omega_h = 2/(2 tau_h + 1),
// coupling factor (1 - omega_h/2)(Pr - 1)/tau_f (Eq. 47).
template <class F>
__device__ __forceinline__ Relax transport(const KArgs &a, real rho, real dth) {
    Relax t;
    if (F_CTAU) {
        t.s_nu = a.s_nu;
        t.s_e = a.s_e;
        t.s_z = a.s_z;
        t.omega_h = a.omega_h;
        t.kcoup = a.kcoup;
        return t;
    }
    const real th = real(1.) + dth;
    real mu3 = a.mu3;
    if (a.visc == LB_VISC_POWER) {
        mu3 *= exp2f(a.visc_n * log2f(a.cT * th));
    } else if (a.visc == LB_VISC_SUTHERLAND) {
        const real r = a.cT * th;
        mu3 *= r * sqrt(r) * (real(1.) + a.sT) * frcp(r + a.sT);
    }
    const real tau = mu3 * frcp(rho * th) + real(0.5);  // p = rho R T = rho theta / 3
    t.s_nu = frcp(tau);
    t.omega_h = real(2.) * a.Pr * frcp(real(2.) * tau - real(1.) + a.Pr);
    t.kcoup = (real(1.) - real(0.5) * t.omega_h) * (a.Pr - real(1.)) * t.s_nu;
    t.s_e = a.tie_e ? t.s_nu : a.s_e;
    t.s_z = a.tie_z ? t.s_nu : a.s_z;
    return t;
}

// Node kind and the node a boundary node extrapolates from (inward normal,
// the diagonal at corners), for the node (x, y) of the domain.
struct BInfo {
    int kind, fx, fy;
    real ux, uy, dth;
};

__device__ __forceinline__ BInfo classify(const KArgs &a, int x, int y) {
    BInfo b;
    b.kind = K_INTERIOR;
    b.fx = x;
    b.fy = y;
    b.ux = b.uy = b.dth = real(0.);
    int hx = -1, hy = -1;
    if (!a.per_x) {
        if (x == 0) hx = 0;
        else if (x == a.nx - 1) hx = 1;
    }
    if (!a.per_y) {
        if (y == 0) hy = 2;
        else if (y == a.ny - 1) hy = 3;
    }
    if (hx < 0 && hy < 0) return b;
    if (hx >= 0) b.fx = (hx == 0) ? 1 : a.nx - 2;
    if (hy >= 0) b.fy = (hy == 2) ? 1 : a.ny - 2;
    if (hx >= 0 && hy >= 0) {
        b.ux = a.side_ux[hx];
        b.uy = a.side_uy[hx];
        if (a.side_kind[hx] == LB_BC_WALL) {
            b.kind = K_DIRICHLET;
            b.dth = a.side_dth[hx];
        } else if (a.side_kind[hy] == LB_BC_WALL) {
            b.kind = K_DIRICHLET;
            b.dth = a.side_dth[hy];
        } else {
            b.kind = K_ADIABATIC;
        }
        return b;
    }
    const int s = hx >= 0 ? hx : hy;
    const int k = a.side_kind[s];
    b.ux = a.side_ux[s];
    b.uy = a.side_uy[s];
    b.dth = a.side_dth[s];
    b.kind = (k == LB_BC_WALL) ? K_DIRICHLET : (k == LB_BC_ADIABATIC) ? K_ADIABATIC : (k == LB_BC_INLET) ? K_INLET : K_OUTLET;
    return b;
}

// The state of node (x, y) at the current time after the boundary treatment
// comes in two parts so that the loads can be issued early: node_issue
// gathers the populations of the node a boundary node extrapolates from (the
// node itself otherwise), node_finish computes the moments and rebuilds the
// populations of boundary nodes.  Returns the node kind.
template <int ST, bool BC>
__device__ __forceinline__ void node_issue(const KArgs &a, const Planes &S, int x, int y, real d[18]) {
    if (!BC) {
        gather<ST>(a, S, x, y, d);
        return;
    }
    const BInfo b = classify(a, x, y);
    gather<ST>(a, S, b.fx, b.fy, d);
}

// On a bounded grid the rebuild runs in FP64 (MomType); a wall node hands its
// FP64 density and temperature deviations to the collision in bw[0], bw[1].
template <int ST, bool BC, class F>
__device__ __forceinline__ int node_finish(const KArgs &a, const Planes &S, int x, int y, real d[18], Mom &m,
                                           double bw[2], unsigned step) {
    typedef typename MomType<kPrecise<ST, BC, F>>::type T;
    m = moments<F>(a, d);
    if (!BC) return K_INTERIOR;
    const BInfo b = classify(a, x, y);
    if (b.kind == K_INTERIOR || b.kind == K_OUTLET) return b.kind;  // outlet: exact copy of the neighbour
    MomT<T> mb;
    if (!F::precise && b.kind == K_INLET) {  // a grid with walls has no inlet
        // s = sin(2 pi n / P) at the time n of the state (Eq. 53): the phase
        // n / P reduced in FP64, the sine in the arithmetic type
        const double t = (double)step * a.in_rate;
        const real s = sin_pi(real(2.) * (real)(t - floor(t)));
        m.drho = a.in_rho * s;
        m.ux = a.in_u * s;
        m.uy = real(0.);
        m.dth = a.in_th * s;
        m.rho = a.rho0 + m.drho;
        m.jx = m.rho * m.ux;
        m.jy = real(0.);
        real he[9];
        equilibria<F>(a, m, d, he);
#pragma unroll
        for (int q = 0; q < 9; ++q) d[9 + q] = he[q];
        const Mom raw = moments<F>(a, d);
        m.sf = raw.sf;
        m.sx = raw.sx;
        m.sy = raw.sy;
        return K_INLET;
    }
    const MomT<T> mf = moments<F, T>(a, d);
    mb.ux = (T)b.ux;
    mb.uy = (T)b.uy;
    if (b.kind == K_DIRICHLET) {
        mb.dth = (T)b.dth;
    } else {
        // T_b = (4 T_1 - T_2) / 3 along the inward normal
        real d2[18];
        gather<ST>(a, S, 2 * b.fx - x, 2 * b.fy - y, d2);
        const MomT<T> m2 = moments<F, T>(a, d2);
        mb.dth = (T(4.) * mf.dth - m2.dth) * (T(1.) / T(3.));
    }
    // pressure extrapolation with the hydrostatic balance of the body force,
    // p_b = p_f exp(x), x = g (y_f - y_b) / (R T_m), T_m = (T_f + T_b)/2
    // (R T0 = 1/3), i.e. rho_b = rho_f theta_f / theta_b (1 + expm1(x));
    // or density extrapolation rho_b = rho_f
    if (a.rho_press) {
        const T x = T(6.) * (T)a.g * (T)(b.fy - y) * frcp(T(2.) + mf.dth + mb.dth);
        const T em1 = x * (T(1.) + x * (T(0.5) + x * (T(1.) / T(6.) + x * (T(1.) / T(24.)))));
        mb.drho = mf.drho + mf.rho * ((mf.dth - mb.dth) + (T(1.) + mf.dth) * em1) * frcp(T(1.) + mb.dth);
    } else {
        mb.drho = mf.drho;
    }
    mb.rho = (T)a.rho0 + mb.drho;
    mb.jx = mb.rho * mb.ux;
    mb.jy = mb.rho * mb.uy;
    T fb[9], hb[9], ff[9], hf[9];
    equilibria<F>(a, mb, fb, hb);
    equilibria<F>(a, mf, ff, hf);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        d[q] = (real)((T)d[q] + (fb[q] - ff[q]));
        d[9 + q] = (real)((T)d[9 + q] + (hb[q] - hf[q]));
    }
    const Mom raw = moments<F>(a, d);
    m = mom_cast<real>(mb);
    m.sf = raw.sf;
    m.sx = raw.sx;
    m.sy = raw.sy;
    bw[0] = (double)mb.drho;
    bw[1] = (double)mb.dth;
    return b.kind;
}

template <int ST, bool BC>
__device__ __forceinline__ int node_state(const KArgs &a, const Planes &S, int x, int y, real d[18], Mom &m) {
    node_issue<ST, BC>(a, S, x, y, d);
    double bw[2];
    return node_finish<ST, BC, Dyn>(a, S, x, y, d, m, bw, a.step);
}

// Collision of one node (Eq. 44 or Eq. 34 for f^, Eq. 47 or Eq. 38 for h-),
// deviations in d, results in o.
// plane_bits: defined with the counter hash below
__device__ __forceinline__ unsigned plane_bits(unsigned h, int q);

// d + inc in FP32 with a rounding that is unbiased on average: inc is dithered
// by a uniform random fraction of one unit in the last place of d before the
// sum rounds to nearest, so that repeated steps of a (nearly) steady state do
// not accumulate the same rounding every step.  (When |inc| < |d| the
// dithered sum rounds down or up with probabilities given by its position
// between the two neighbours of the exact sum.)
__device__ __forceinline__ float add_dithered(float d, float inc, unsigned bits) {
    const float u = __uint_as_float(__float_as_uint(d) & 0x7f800000u) * 0x1p-23f;  // ulp of d (0 for 0)
    const float r = __uint_as_float(0x3f800000u | (bits >> 9)) - 1.5f;               // uniform in [-1/2, 1/2)
    return d + fmaf(r, u, inc);
}
#ifdef LB_ARITH_FP64
__device__ __forceinline__ double add_dithered(double d, double inc, unsigned) { return d + inc; }
#endif

// The moment-space increments (Eq. 44) are formed in the moment type of the
// grid (MomType), then applied in the arithmetic type.  On a bounded grid the
// FP64 moments are the sums of the populations, except that a wall node takes
// its FP64 density and temperature (bw) and its wall velocity.
template <class F, bool PR>
__device__ __forceinline__ void collide(const KArgs &a, const real d[18], const Mom &m, int kind, const double bw[2],
                                        real phix, real phiy, real o[18], unsigned rb) {
    typedef typename MomType<PR>::type T;
    MomT<T> mt = moments<F, T>(a, d);
    if (PR && (kind == K_DIRICHLET || kind == K_ADIABATIC)) {
        mt.drho = (T)bw[0];
        mt.dth = (T)bw[1];
        mt.rho = (T)a.rho0 + mt.drho;
        mt.ux = (T)m.ux;
        mt.uy = (T)m.uy;
        mt.jx = mt.rho * mt.ux;
        mt.jy = mt.rho * mt.uy;
    }
    if (!PR) mt = mom_cast<T>(m);
    // FP32 equilibria: the h update of the FP32 path and the inlet (a grid
    // with walls has no inlet, and its h update runs in the moment type)
    real fe[9], he[9];
    if (!PR) equilibria<F>(a, m, fe, he);
    if (!PR && kind == K_INLET) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            o[q] = fe[q];
            o[9 + q] = he[q];
        }
        return;
    }
    const Relax t = transport<F>(a, m.rho, m.dth);
    const real ux = m.ux, uy = m.uy;
    const real ay = -m.rho * a.g;
    // velocity-space sources C = M^-1 (C^ + F^): Eq. 49 plus the forcing term
    const real w0 = real(4.) / real(9.), w1 = real(1.) / real(9.), w2 = real(1.) / real(36.);
    real C[9];
    {
        const real cx0 = -phix * (real(1.) / real(9.)), cx1 = -phix * (real(1.) / real(36.)), cx2 = phix * (real(1.) / real(18.));
        const real cy = real(0.25) * phiy;
        C[0] = cx0;
        C[1] = C[3] = cx1 + cy;
        C[2] = C[4] = cx1 - cy;
        C[5] = C[6] = C[7] = C[8] = cx2;
        if (F_FORCE) {
            const real f3 = -real(3.) * uy * ay;
            C[0] += w0 * f3;
            C[1] += w1 * f3;
            C[3] += w1 * f3;
            C[2] += w1 * ay * (real(3.) + real(6.) * uy);
            C[4] += w1 * ay * (-real(3.) + real(6.) * uy);
            C[5] += w2 * ay * (real(3.) + real(9.) * ux + real(6.) * uy);
            C[6] += w2 * ay * (real(3.) - real(9.) * ux + real(6.) * uy);
            C[7] += w2 * ay * (-real(3.) + real(9.) * ux + real(6.) * uy);
            C[8] += w2 * ay * (-real(3.) - real(9.) * ux + real(6.) * uy);
        }
    }
    {
        // BGK (Eq. 34) is the MRT scheme with every rate equal to 1/tau_f, so both
        // run through the same moment-space increments.
        const T sr = (T)(F_BGK ? t.s_nu : a.s_rho), sj = (T)(F_BGK ? t.s_nu : a.s_j);
        const T se = (T)(F_BGK ? t.s_nu : t.s_e), sz = (T)(F_BGK ? t.s_nu : t.s_z);
        const T sq = (T)(F_BGK ? t.s_nu : a.s_q), sn = (T)t.s_nu;
        T dt[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) dt[q] = (T)d[q];
        // moments of the deviations, m = M f (Eq. B1); the conserved ones are
        // the raw sums, so that their increments vanish exactly on interior nodes
        const T s1 = (dt[1] + dt[3]) + (dt[2] + dt[4]);
        const T s2 = (dt[5] + dt[7]) + (dt[6] + dt[8]);
        const T dx13 = dt[1] - dt[3], dy24 = dt[2] - dt[4];
        const T a57 = dt[5] - dt[7], a86 = dt[8] - dt[6], a68 = dt[6] - dt[8];
        const T m1 = -T(4.) * dt[0] - s1 + T(2.) * s2;
        const T m2 = T(4.) * dt[0] - T(2.) * s1 + s2;
        const T m4 = -T(2.) * dx13 + (a57 + a86);
        const T m6 = -T(2.) * dy24 + (a57 + a68);
        const T m7 = (dt[1] + dt[3]) - (dt[2] + dt[4]);
        const T m8 = (dt[5] + dt[7]) - (dt[6] + dt[8]);
        // equilibria Eq. 41 minus M f_rest
        const T thE = F_COUPLED ? mt.dth : T(0.);
        const T uxt = mt.ux, uyt = mt.uy, ayt = -mt.rho * (T)a.g;
        const T qq = T(3.) * (mt.jx * uxt + mt.jy * uyt) + T(2.) * mt.rho * thE;
        const T e1 = -T(2.) * mt.drho + qq, e2 = mt.drho - qq;
        const T e4 = -mt.jx * (T(1.) - thE), e6 = -mt.jy * (T(1.) - thE);
        const T e7 = mt.jx * uxt - mt.jy * uyt, e8 = mt.jx * uyt;
        // sources C^ = (0, phi_x, 0, 0, 0, 0, 0, phi_y, 0) + F^ (Eq. 48, 51)
        const T uay = uyt * ayt;
        const T c1 = (T)phix + T(6.) * uay, c2 = -T(6.) * uay, c5 = ayt, c6 = -ayt, c7 = (T)phiy - T(2.) * uay,
                c8 = uxt * ayt;
        // Eq. 44 as increments dm = m* - m
        const real g0 = (real)(-sr * (mt.sf - mt.drho));
        const real g1 = (real)(-se * (m1 - e1) + (T(1.) - T(0.5) * se) * c1);
        const real g2 = (real)(-sz * (m2 - e2) + (T(1.) - T(0.5) * sz) * c2);
        const real g3 = (real)(-sj * (mt.sx - mt.jx));
        const real g4 = (real)(-sq * (m4 - e4));
        const real g5 = (real)(-sj * (mt.sy - mt.jy) + (T(1.) - T(0.5) * sj) * c5);
        const real g6 = (real)(-sq * (m6 - e6) + (T(1.) - T(0.5) * sq) * c6);
        const real g7 = (real)(-sn * (m7 - e7) + (T(1.) - T(0.5) * sn) * c7);
        const real g8 = (real)(-sn * (m8 - e8) + (T(1.) - T(0.5) * sn) * c8);
        // f* = f + M^-1 dm (Eq. B2)
        const real A = g0 * (real(1.) / real(9.));
        const real a1 = A - g1 * (real(1.) / real(36.)) - g2 * (real(1.) / real(18.));
        const real a2 = A + g1 * (real(1.) / real(18.)) + g2 * (real(1.) / real(36.));
        const real X = (g3 - g4) * (real(1.) / real(6.)), Y = (g5 - g6) * (real(1.) / real(6.)), P = real(0.25) * g7;
        const real X2 = g3 * (real(1.) / real(6.)) + g4 * (real(1.) / real(12.)), Y2 = g5 * (real(1.) / real(6.)) + g6 * (real(1.) / real(12.));
        const real Pxy = real(0.25) * g8;
        o[0] = (PR && a.dither) ? add_dithered(d[0], (A + (g2 - g1) * (real(1.) / real(9.))), plane_bits(rb, 0)) : d[0] + (A + (g2 - g1) * (real(1.) / real(9.)));
        o[1] = (PR && a.dither) ? add_dithered(d[1], (a1 + X + P), plane_bits(rb, 1)) : d[1] + (a1 + X + P);
        o[3] = (PR && a.dither) ? add_dithered(d[3], (a1 - X + P), plane_bits(rb, 3)) : d[3] + (a1 - X + P);
        o[2] = (PR && a.dither) ? add_dithered(d[2], (a1 + Y - P), plane_bits(rb, 2)) : d[2] + (a1 + Y - P);
        o[4] = (PR && a.dither) ? add_dithered(d[4], (a1 - Y - P), plane_bits(rb, 4)) : d[4] + (a1 - Y - P);
        o[5] = (PR && a.dither) ? add_dithered(d[5], (a2 + X2 + Y2 + Pxy), plane_bits(rb, 5)) : d[5] + (a2 + X2 + Y2 + Pxy);
        o[6] = (PR && a.dither) ? add_dithered(d[6], (a2 - X2 + Y2 - Pxy), plane_bits(rb, 6)) : d[6] + (a2 - X2 + Y2 - Pxy);
        o[7] = (PR && a.dither) ? add_dithered(d[7], (a2 - X2 - Y2 + Pxy), plane_bits(rb, 7)) : d[7] + (a2 - X2 - Y2 + Pxy);
        o[8] = (PR && a.dither) ? add_dithered(d[8], (a2 + X2 - Y2 - Pxy), plane_bits(rb, 8)) : d[8] + (a2 + X2 - Y2 - Pxy);
    }
    // h: BGK plus the coupling term (1 - omega_h/2)(Z/tau_hf)(f - f_eq + C/2), Z = e.u
    if (PR) {
        // in the moment type: the equilibria and the non-equilibrium h - h_eq
        // of O(1) deviations, with the same closure of the zeroth moment
        T fT[9], hT[9];
        equilibria<F>(a, mt, fT, hT);
        T dh[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) dh[q] = (T)d[9 + q];
        hT[0] = (((dh[0] + dh[1]) + (dh[2] + dh[3])) + ((dh[4] + dh[5]) + (dh[6] + dh[7])) + dh[8]) -
                (((hT[1] + hT[2]) + (hT[3] + hT[4])) + ((hT[5] + hT[6]) + (hT[7] + hT[8])));
        const T whT = (T)t.omega_h, kT = (T)t.kcoup;
        const T v5 = mt.ux + mt.uy, v6 = mt.uy - mt.ux;
        const T z[9] = {T(0.), mt.ux, mt.uy, -mt.ux, -mt.uy, v5, v6, -v5, -v6};
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            T inc = -whT * (dh[q] - hT[q]);
            if (F_HEAT && q > 0) inc += kT * z[q] * ((T)d[q] - fT[q] + T(0.5) * (T)C[q]);
            o[9 + q] = a.dither ? add_dithered(d[9 + q], (real)inc, plane_bits(rb, 9 + q)) : d[9 + q] + (real)inc;
        }
        return;
    }
    // The zeroth moment of h_eq must equal the energy of the node, i.e. the raw
    // sum of its h, so that the BGK relaxation of h conserves energy.  The
    // weights 4/9, 1/9, 1/36 are not representable in binary and round with
    // one common relative error (about +7e-9 in FP32): the plain sum would
    // add that fraction of the local energy deviation every step, a steady
    // heat source that follows the gravity stratification and biases the
    // flow.  h_eq of the rest velocity absorbs the remainder.
    he[0] = (((d[9] + d[10]) + (d[11] + d[12])) + ((d[13] + d[14]) + (d[15] + d[16])) + d[17]) -
            (((he[1] + he[2]) + (he[3] + he[4])) + ((he[5] + he[6]) + (he[7] + he[8])));
    const real wh = t.omega_h;
#pragma unroll
    for (int q = 0; q < 9; ++q) o[9 + q] = d[9 + q] - wh * (d[9 + q] - he[q]);
    if (F_HEAT) {
        const real k = t.kcoup;
        const real v5 = ux + uy, v6 = uy - ux;
        const real z[9] = {real(0.), ux, uy, -ux, -uy, v5, v6, -v5, -v6};
#pragma unroll
        for (int q = 1; q < 9; ++q) o[9 + q] += k * z[q] * (d[q] - fe[q] + real(0.5) * C[q]);
    }
}

// Counter-based random bits for the stochastic rounding of the 16-bit codecs
// and the dithered FP32 sums: a 32-bit integer hash of the node's linear
// index and the time step, rotated by a different amount for each of the 18
// planes so that each plane's rounding reads a different window of it.  The
// hash is "lowbias32" (two multiply-xorshift rounds, multipliers 0x7feb352d
// and 0x846ca68b), found by C. Wellons' hash-prospector search and published
// with it.
__device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ unsigned plane_bits(unsigned h, int q) {
    return __builtin_amdgcn_alignbit(h, h, (7u * (unsigned)q) & 31u);
}

__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3, per = nb >> 3, rem = nb & 7;
    return xcd * per + min(xcd, rem) + idx;
}

// Rows of the marching strip: y may be -1 or ny.  A periodic axis wraps; a
// bounded one clamps (those rows only feed Q, which is then zero, to
// boundary nodes, whose correction term is zero anyway).
__device__ __forceinline__ int row_wrap(const KArgs &a, int y, bool &yin) {
    if (a.per_y) {
        yin = true;
        return y < 0 ? y + a.ny : (y >= a.ny ? y - a.ny : y);
    }
    yin = (y >= 0) && (y < a.ny);
    return min(max(y, 0), a.ny - 1);
}

template <int ST, bool BC>
__device__ __forceinline__ void row_issue(const KArgs &a, const Planes &S, int xw, int y, real d[18]) {
    bool yin;
    const int yw = row_wrap(a, y, yin);
    if (BC && !yin) return;  // outside a bounded axis: only its Q (zero) is used
    node_issue<ST, BC>(a, S, xw, yw, d);
}

// Moments, kind and Q = rho u (1 - theta) (Eq. 48) of the lane's node in row y.
template <int ST, bool BC, class F>
__device__ __forceinline__ int row_finish(const KArgs &a, const Planes &S, int xw, bool xin, int y, real d[18],
                                          Mom &m, double bw[2], real &Qx, real &Qy, unsigned step) {
    bool yin;
    const int yw = row_wrap(a, y, yin);
    if (BC && !yin) {
        // a row outside a bounded axis feeds only Q_y to the boundary row
        // next to it, whose correction term is zero
        Qx = Qy = real(0.);
        return K_INTERIOR;
    }
    const int kind = node_finish<ST, BC, F>(a, S, xw, yw, d, m, bw, step);
    const real mq = (F_CORR && xin && yin) ? -m.rho * m.dth : real(0.);
    Qx = mq * m.ux;
    Qy = mq * m.uy;
    return kind;
}

// Correction term from the Q of the neighbours (Eq. 50: central differences;
// x-neighbours from the adjacent lanes, the two tile-edge neighbours from the
// halo values qhl, qhr), collision, store of the owned lanes.
template <int ST, bool BC, class F>
__device__ __forceinline__ void collide_store(const KArgs &a, const Planes &D, const real d[18], const Mom &m,
                                              const double bw[2],
                                              int kind, int lane, real qxc, real qhl, real qhr, real qyp,
                                              real qyn, bool owned, unsigned vo, unsigned step) {
    real qxl = __shfl_up(qxc, 1), qxr = __shfl_down(qxc, 1);
    qxl = lane == 0 ? qhl : qxl;
    qxr = lane == kWave - 1 ? qhr : qxr;
    const real dQx = real(0.5) * (qxr - qxl), dQy = real(0.5) * (qyn - qyp);
    real phix = real(3.) * (dQx + dQy), phiy = dQx - dQy;
    if (BC && kind != K_INTERIOR) phix = phiy = real(0.);
    real o[18];
    // random bits of the node and step: the stochastic rounding of the 16-bit
    // codecs and of the FP64-arithmetic library's FP32 stores, the dithered
    // sums of the bounded FP32 step
#ifdef LB_ARITH_FP64
    constexpr bool need_bits = true;
#else
    constexpr bool need_bits = ST != LB_STORE_F32 || kPrecise<ST, BC, F>;
#endif
    const unsigned h = need_bits ? hash32((vo / Codec<ST>::bytes) ^ (step * 0x9E3779B9u)) : 0u;
    collide<F, kPrecise<ST, BC, F>>(a, d, m, kind, bw, phix, phiy, o, h);
    if (owned) {
#pragma unroll
        for (int q = 0; q < 18; ++q) Codec<ST>::st(D, vo, o[q], q, plane_bits(h, q));
    }
}

// lane's column x of a tile, wrapped (periodic) or clamped (bounded); xin
// tells whether x lies inside the domain.
__device__ __forceinline__ int col_wrap(const KArgs &a, int x, bool &xin) {
    if (a.per_x) {
        xin = true;
        int xw = x % a.nx;
        return xw + ((xw < 0) ? a.nx : 0);
    }
    xin = (x >= 0) && (x < a.nx);
    return min(max(x, 0), a.nx - 1);
}

// x-component of Q (Eq. 48) at the two columns just outside the wavefront's
// tile for up to 32 rows of the strip's march from row yb (direction dir):
// lanes 0..31 take column x0 - 1, lanes 32..63 column x0 + 64, row
// yb + dir (lane & 31); lanes past the strip's end repeat its last row and go
// unused, and a side that is not needed is skipped.  One wide gather thus
// serves 32 rows; the row loop picks its values out with readlane.  The
// gather is split into the issue of its loads and the finish, so that the
// strip's first chunk is in flight together with its first rows.
struct HaloPos {
    int xw, y;
    bool xin, on;
};

__device__ __forceinline__ HaloPos halo_pos(const KArgs &a, int x0, int lane, int yb, int dir, int ylo, int yhi,
                                            bool need_l, bool need_r) {
    const bool left = lane < kHaloRows;
    HaloPos h;
    h.on = left ? need_l : need_r;
    h.xw = col_wrap(a, left ? x0 - 1 : x0 + kTile, h.xin);
    h.y = min(max(yb + dir * (lane & (kHaloRows - 1)), ylo), yhi);
    return h;
}

template <int ST, bool BC>
__device__ __forceinline__ void halo_issue(const KArgs &a, const Planes &S, const HaloPos &h, real dh[18]) {
    if (h.on) row_issue<ST, BC>(a, S, h.xw, h.y, dh);
}

template <int ST, bool BC, class F>
__device__ __forceinline__ real halo_finish(const KArgs &a, const Planes &S, const HaloPos &h, real dh[18],
                                            unsigned step) {
    real qx = real(0.);
    if (h.on) {
        Mom mh;
        double bwh[2];
        real qy;
        row_finish<ST, BC, F>(a, S, h.xw, h.xin, h.y, dh, mh, bwh, qx, qy, step);
    }
    return qx;
}

template <int ST, bool BC, class F>
__device__ __forceinline__ real halo_chunk(const KArgs &a, const Planes &S, int x0, int lane, int yb, int dir,
                                            int ylo, int yhi, bool need_l, bool need_r, unsigned step) {
    const HaloPos h = halo_pos(a, x0, lane, yb, dir, ylo, yhi, need_l, need_r);
    real dh[18];
    halo_issue<ST, BC>(a, S, h, dh);
    return halo_finish<ST, BC, F>(a, S, h, dh, step);
}

// One strip: LW wavefronts side by side, wavefront w owning the 64 aligned
// columns from x0 = 64 tx (tx = its tile), all of them marching through rows
// [R sy, R sy + R) in step: up on even strips, down on odd ones, so that two
// neighbouring strips reach the rows they share (each reads two rows of the
// other) at the same moment, both at their start or both at their end, while
// those rows are still in L2.  With LW > 1 the block's wavefronts are
// adjacent tiles: each row they meet at one barrier and pass the Q_x of their
// edge lanes to their neighbours through LDS, so only the two outer
// wavefronts gather halo columns, and the cache lines that neighbouring tiles
// share are fetched by both at the same time.  LW = 1 is the packed (serving)
// step, where every wavefront runs on its own.
template <int ST, bool BC, class F, int LW>
__device__ __forceinline__ void run_strip(const KArgs &a, const char *__restrict__ src, char *__restrict__ dst,
                                          int tx, int sy, unsigned step) {
    // Q_x of the edge lanes (0: lane 0, 1: lane 63) of each wavefront, three
    // row slots so that one barrier per row separates writes from reads
    __shared__ real qedge[3][LW][2];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = LW > 1 ? (int)(threadIdx.x >> 6) : 0;
    const bool edge_l = w == 0, edge_r = w == LW - 1;
    const int wl = max(w - 1, 0), wr = min(w + 1, LW - 1);
    const int x0 = tx * kTile, gx = x0 + lane;
    bool xin;
    const int xw = col_wrap(a, gx, xin);
    const bool owned = gx < a.nx;
    const int y0 = sy * a.strip_rows;
    const int y1 = min(y0 + a.strip_rows, a.ny);
    const int dir = (sy & 1) ? -1 : 1;
    const int ys = dir > 0 ? y0 : y1 - 1;  // first row of the march
    const Planes S = planes(src, a), D = planes(dst, a);
    const unsigned eb = Codec<ST>::bytes;
    const unsigned dvo = (unsigned)(dir * a.rs) * eb;  // store offset step (wraps for dir < 0)
    unsigned vo = ((unsigned)ys * a.rs + xw) * eb;

    // halo Q_x from the gathered chunk (outer wavefronts only; a column
    // outside a bounded axis has Q = 0 and is not gathered)
    const bool need_l = edge_l && (a.per_x || x0 > 0), need_r = edge_r && (a.per_x || x0 + kTile < a.nx);

    // two row states used alternately (the loop is unrolled by two); qyb is
    // Q_y of the row behind the current one
    real dA[18], dB[18];
    Mom mA, mB;
    double bwA[2], bwB[2];  // FP64 wall values (bounded grids)
    real qyb, qxA, qyA, qxB, qyB;
    // the first halo chunk, the row behind the first and the first row: all
    // their loads in flight at once (a short strip is bound by their latency)
    const HaloPos hp = halo_pos(a, x0, lane, ys, dir, y0, y1 - 1, need_l, need_r);
    real qh;
    {
        real dh[18];
        halo_issue<ST, BC>(a, S, hp, dh);
        row_issue<ST, BC>(a, S, xw, ys - dir, dB);
        row_issue<ST, BC>(a, S, xw, ys, dA);
        qh = halo_finish<ST, BC, F>(a, S, hp, dh, step);
    }
    row_finish<ST, BC, F>(a, S, xw, xin, ys - dir, dB, mB, bwB, qxB, qyb, step);
    int kA = row_finish<ST, BC, F>(a, S, xw, xin, ys, dA, mA, bwA, qxA, qyA, step), kB;
    int sc = 0;  // LDS slot of the current row
    if (LW > 1) {
        if (lane == 0) qedge[0][w][0] = qxA;
        if (lane == kWave - 1) qedge[0][w][1] = qxA;
    }

    // One row (k rows into the march): issue the look-ahead row's loads,
    // finish it, publish its edge Q_x, then collide and store the current row.
    auto row = [&](int k, real(&dC)[18], const Mom &mC, const double(&bwC)[2], int kC, real qxC, real(&dN)[18],
                   Mom &mN, double(&bwN)[2], int &kN, real &qxN, real &qyN) {
        const int y = ys + dir * k;
        row_issue<ST, BC>(a, S, xw, y + dir, dN);
        const int r = k & (kHaloRows - 1);
        if ((need_l || need_r) && r == 0 && k != 0)
            qh = halo_chunk<ST, BC, F>(a, S, x0, lane, y, dir, y0, y1 - 1, need_l, need_r, step);
        real qhl = readlane_real(qh, r);
        real qhr = readlane_real(qh, kHaloRows + r);
        kN = row_finish<ST, BC, F>(a, S, xw, xin, y + dir, dN, mN, bwN, qxN, qyN, step);
        if (LW > 1) {
            const int sn = sc == 2 ? 0 : sc + 1;
            if (lane == 0) qedge[sn][w][0] = qxN;
            if (lane == kWave - 1) qedge[sn][w][1] = qxN;
            __syncthreads();
            if (!edge_l) qhl = qedge[sc][wl][1];
            if (!edge_r) qhr = qedge[sc][wr][0];
            sc = sn;
        }
        // Q_y at y - 1 and y + 1
        const real qym = dir > 0 ? qyb : qyN, qyq = dir > 0 ? qyN : qyb;
        collide_store<ST, BC, F>(a, D, dC, mC, bwC, kC, lane, qxC, qhl, qhr, qym, qyq, owned, vo, step);
        vo += dvo;
    };
    const int rows = y1 - y0;
    int k = 0;
    for (;;) {
        if (k >= rows) break;
        row(k, dA, mA, bwA, kA, qxA, dB, mB, bwB, kB, qxB, qyB);
        qyb = qyA;
        ++k;
        if (k >= rows) break;
        row(k, dB, mB, bwB, kB, qxB, dA, mA, bwA, kA, qxA, qyA);
        qyb = qyB;
        ++k;
    }
}

// ----------------------------------------------------------------- kernels
// Block = kLock wavefronts on adjacent tiles of one strip (see run_strip).
// The time step of the state read is clk[0] + sub when clk is given (the
// launches of a captured k-step graph, whose arguments are fixed), else
// a.step + sub.
template <int ST, bool BC, class F>
__global__ __launch_bounds__(kWave * kLock<ST>) void k_step(const KArgs a, const char *__restrict__ src,
                                                            char *__restrict__ dst, const long long *__restrict__ clk,
                                                            int sub) {
    constexpr int LW = kLock<ST>;
    const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
    const int bxs = (a.tiles_x + LW - 1) / LW;
    const int bx = blk % bxs, sy = blk / bxs;
    const unsigned step = (unsigned)((clk ? clk[0] : (long long)a.step) + sub);
    run_strip<ST, BC, F, LW>(a, src, dst, bx * LW + (int)(threadIdx.x >> 6), sy, step);
}

// Sets the step clock that the launches of a captured graph read.
__global__ void k_set_clock(long long *clk, long long n) { clk[0] = n; }

// Packed step of many grids (serving).  The work list has two parts: the
// items of the grids in the cavity configuration, stepped by a launch of the
// kernel specialised for it (CavW), then those of the other grids (DynW), by
// a launch of the general one; a grid's kernel follows from its own switches,
// so its arithmetic does not depend on the mix.  Within a part come, first,
// the block items of the wide grids (FP32 storage, at least kWavesPerBlock
// tiles across): a block runs kWavesPerBlock adjacent tiles of one strip in
// lockstep, as the single-grid step does; then the wavefront items of the
// narrow grids (all grids of the 16-bit codecs), one tile of one strip each,
// run by the wavefronts of a block independently.  One kernel, a fixed grid
// of blocks numbered XCD by XCD so that runs of neighbouring items share an
// L2, goes over its part in rounds: the wide grids' items first, then the
// narrow ones four to a block.  A grid is always wide or always narrow.  Call
// i of a batch reads buffer (cur + i) & 1 of each grid.
struct SlotDev {
    KArgs a;
    const char *pops[2];
    int cur, pad_;
    long long n;  // time step at the start of the batch
};
struct WorkItem {
    int slot, tx, sy, pad_;
};

// 2 wavefronts per SIMD with FP32 storage, whose served grids (all bounded)
// form their moments in FP64 and carry both the wide and the narrow path; 3
// for the 16-bit codecs, which have the narrow path only (measured: the wide
// one made their packed step slower).
template <int ST>
constexpr int kMultiWaves = ST == LB_STORE_F32 ? 2 : 3;

// counts = {wide, narrow items of part 0, wide, narrow items of part 1}; the
// items of part 1 follow those of part 0.
template <int ST, class F>
__global__ __launch_bounds__(kBlock, kMultiWaves<ST>) void k_step_multi(const SlotDev *__restrict__ slots,
                                                                         const WorkItem *__restrict__ items,
                                                                         const int *__restrict__ counts, int part,
                                                                         int i) {
    const int nwide = counts[2 * part], nnarrow = counts[2 * part + 1];
    if (part) items += counts[0] + counts[1];
    const int nblk = nwide + (nnarrow + kWavesPerBlock - 1) / kWavesPerBlock;
    const int wv = (int)(threadIdx.x >> 6);
    // Rounds of gridDim.x block items; in each, the m blocks that have one
    // take consecutive items XCD by XCD (m may be far below gridDim.x: the
    // items must not be packed onto the first XCDs).  b is the same on every
    // thread of the block, so both branches and the barriers in the wide one
    // are block-uniform.
    for (int r0 = 0; r0 < nblk; r0 += gridDim.x) {
        const int m = min((int)gridDim.x, nblk - r0);
        if ((int)blockIdx.x >= m) break;  // only the last round is short
        const int b = r0 + xcd_swizzle(blockIdx.x, m);
        if (ST == LB_STORE_F32 && b < nwide) {
            const WorkItem it = items[b];
            const SlotDev &sd = slots[it.slot];
            const int c = (sd.cur + i) & 1;
            run_strip<ST, true, F, kWavesPerBlock>(sd.a, sd.pops[c], const_cast<char *>(sd.pops[c ^ 1]), it.tx + wv,
                                                  it.sy, (unsigned)(sd.n + i));
            __syncthreads();  // the next item rewrites the LDS edge slots
        } else {
            // the item index is the same on every lane of the wavefront:
            // readfirstlane lets the compiler load the item and its grid's
            // arguments with scalar loads instead of once per lane
            const int w = __builtin_amdgcn_readfirstlane(nwide + (b - nwide) * kWavesPerBlock + wv);
            if (w < nwide + nnarrow) {
                const WorkItem it = items[w];
                const SlotDev &sd = slots[it.slot];
                const int c = (sd.cur + i) & 1;
                run_strip<ST, true, F, 1>(sd.a, sd.pops[c], const_cast<char *>(sd.pops[c ^ 1]), it.tx, it.sy,
                                         (unsigned)(sd.n + i));
            }
        }
    }
}

// Initial state: the pull of the first step must see the equilibria of the
// fields, so node (x, y) writes its equilibria to (x, y) - e_a.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_init(const KArgs a, const float *__restrict__ fields, long long fplane,
                                                 char *__restrict__ dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.nx * a.ny) return;
    const int x = i % a.nx, y = i / a.nx;
    const unsigned k = (unsigned)y * a.pitch + x;
    Mom m;
    m.drho = fields[k];
    m.ux = fields[fplane + k];
    m.uy = fields[2 * fplane + k];
    m.dth = fields[3 * fplane + k];
    m.rho = a.rho0 + m.drho;
    m.jx = m.rho * m.ux;
    m.jy = m.rho * m.uy;
    m.sf = m.sx = m.sy = real(0.);
    real fe[9], he[9];
    equilibria<Dyn>(a, m, fe, he);
    const Planes D = planes(dst, a);
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        int tx = x - ex[q], ty = y - ey[q];
        if (tx < 0 || tx >= a.nx) {
            if (!a.per_x) continue;
            tx += (tx < 0) ? a.nx : -a.nx;
        }
        if (ty < 0 || ty >= a.ny) {
            if (!a.per_y) continue;
            ty += (ty < 0) ? a.ny : -a.ny;
        }
        const unsigned t = ((unsigned)ty * a.rs + tx) * Codec<ST>::bytes;
        Codec<ST>::st(D, t, fe[q], q, plane_bits(hash32(t ^ 0x5bd1e995u), q));
        Codec<ST>::st(D, t, he[q], 9 + q, plane_bits(hash32(t ^ 0x5bd1e995u), 9 + q));
    }
}

// Moments (deviations drho, ux, uy, dtheta) after the boundary treatment.
// full != 0 writes rho and T = T0 theta with T0 = tscale instead.
template <int ST, bool BC>
__global__ __launch_bounds__(kBlock) void k_macros(const KArgs a, const char *__restrict__ src, float *__restrict__ o0,
                                                   float *__restrict__ o1, float *__restrict__ o2,
                                                   float *__restrict__ o3, int opitch, int full, real tscale) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.nx * a.ny) return;
    const int x = i % a.nx, y = i / a.nx;
    real d[18];
    Mom m;
    node_state<ST, BC>(a, planes(src, a), x, y, d, m);
    const unsigned k = (unsigned)y * opitch + x;
    if (o0) o0[k] = full ? m.rho : m.drho;
    if (o1) o1[k] = m.ux;
    if (o2) o2[k] = m.uy;
    if (o3) o3[k] = full ? tscale * (real(1.) + m.dth) : m.dth;
}

// Population deviations after the boundary treatment, planes q0 .. q0+nq-1.
template <int ST, bool BC>
__global__ __launch_bounds__(kBlock) void k_pops(const KArgs a, const char *__restrict__ src, float *__restrict__ out,
                                                 long long oplane, int q0, int nq) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.nx * a.ny) return;
    const int x = i % a.nx, y = i / a.nx;
    real d[18];
    Mom m;
    node_state<ST, BC>(a, planes(src, a), x, y, d, m);
    const unsigned k = (unsigned)y * a.pitch + x;
#pragma unroll
    for (int q = 0; q < 18; ++q)
        if (q >= q0 && q < q0 + nq) out[(q - q0) * oplane + k] = d[q];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// FP64 sums over the grid: [sum d_f, sum d_h, sum e_x d_f, sum e_y d_f, #bad,
// sum (dth - snap)^2, sum (1 + dth)^2, 0] as per-block partials.
template <int ST, bool BC>
__global__ __launch_bounds__(kBlock) void k_diag(const KArgs a, const char *__restrict__ src, float *__restrict__ snap,
                                                 int use_snap, int write_snap, double *__restrict__ partials) {
    double acc[kNred] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int n = a.nx * a.ny;
    const Planes P = planes(src, a);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int x = i % a.nx, y = i / a.nx;
        real d[18];
        Mom m;
        node_state<ST, BC>(a, P, x, y, d, m);
        double sf = 0, sh = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            sf += (double)d[q];
            sh += (double)d[9 + q];
        }
        acc[0] += sf;
        acc[1] += sh;
        acc[2] += ((double)d[1] - d[3]) + ((double)d[5] - d[6]) + ((double)d[8] - d[7]);
        acc[3] += ((double)d[2] - d[4]) + ((double)d[5] + d[6]) - ((double)d[7] + d[8]);
        const bool ok = isfinite(m.rho) && isfinite(m.ux) && isfinite(m.uy) && isfinite(m.dth) && m.rho > real(0.) &&
                        (real(1.) + m.dth) > real(0.);
        acc[4] += ok ? 0.0 : 1.0;
        const unsigned k = (unsigned)y * a.pitch + x;
        if (use_snap) {
            const double e = (double)m.dth - (double)snap[k];
            acc[5] += e * e;
        }
        const double t = 1.0 + (double)m.dth;
        acc[6] += t * t;
        if (write_snap) snap[k] = m.dth;
    }
    __shared__ double red[kNred][kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kNred; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) red[j][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNred) {
        double s = 0;
        for (int j = 0; j < kWavesPerBlock; ++j) s += red[threadIdx.x][j];
        partials[blockIdx.x * kNred + threadIdx.x] = s;
    }
}

// Sum j of the per-block partials in a fixed order, returned on thread j
// (j < kNred) of the one block.
__device__ __forceinline__ double reduce_partials(const double *__restrict__ partials, int nblocks) {
    __shared__ double red[kNred][kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    for (int j = 0; j < kNred; ++j) {
        double s = 0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[b * kNred + j];
        s = wave_sum(s);
        if (lane == 0) red[j][w] = s;
    }
    __syncthreads();
    double s = 0;
    if (threadIdx.x < kNred)
        for (int j = 0; j < kWavesPerBlock; ++j) s += red[threadIdx.x][j];
    return s;
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(const double *__restrict__ partials, int nblocks,
                                                         double *__restrict__ out) {
    const double s = reduce_partials(partials, nblocks);
    if (threadIdx.x < kNred) out[threadIdx.x] = s;
}

// The diagnostics of lb_diag on the device: out[0] = base_f + sum d_f,
// out[1] = base_h + sum d_h, out[2..4] the momentum sums and the bad-node
// count, out[5] = time step.
__global__ __launch_bounds__(kBlock) void k_diag_final(const double *__restrict__ partials, int nblocks, double base_f,
                                                       double base_h, double time, double *__restrict__ out) {
    const double s = reduce_partials(partials, nblocks);
    if (threadIdx.x < 5) out[threadIdx.x] = threadIdx.x == 0 ? base_f + s : (threadIdx.x == 1 ? base_h + s : s);
    if (threadIdx.x == 5) out[5] = time;
}

// STREAM-like copy of n 16-byte vectors: the practical memory ceiling that
// the step's bandwidth is compared with.  Block b copies the contiguous
// vectors [b chunk, min(n, (b + 1) chunk)), four loads in flight per lane
// before their non-temporal stores (measured on 2 GiB: 5.4 TB/s; lanes
// striding over the whole buffer reached 4.5-4.9 TB/s).
typedef unsigned V4u __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(kBlock) void k_copy(const V4u *__restrict__ src, V4u *__restrict__ dst, long long n,
                                                 long long chunk) {
    constexpr int U = kCopyUnroll;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    long long i = lo + threadIdx.x;
    for (; i + (U - 1) * kBlock < hi; i += U * kBlock) {
        V4u v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[i + u * kBlock];
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * kBlock]);
    }
    for (; i < hi; i += kBlock) __builtin_nontemporal_store(src[i], &dst[i]);
}

// ------------------------------------------------------------- host side
thread_local std::string g_err;

lb_status fail(lb_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    int pitch;
    size_t plane_elems, plane_bytes, pops_bytes, snap_off, snap_bytes, part_off, red_off, clk_off, total;
    int ssize;
};

Layout layout_of(const lb_params *p) {
    Layout L;
    L.ssize = p->storage == LB_STORE_F32 ? 4 : 2;
    L.pitch = (int)align_up((size_t)p->nx, 64);
    L.plane_elems = (size_t)L.pitch * p->ny + kPlanePadBytes / L.ssize;  // one population's rows
    L.plane_bytes = L.plane_elems * L.ssize;
    L.pops_bytes = align_up(18 * L.plane_bytes, 256);
    L.snap_off = 2 * L.pops_bytes;
    L.snap_bytes = align_up((size_t)L.pitch * p->ny * sizeof(float), 256);
    L.part_off = L.snap_off + L.snap_bytes;
    L.red_off = L.part_off + align_up(kRedBlocks * kNred * sizeof(double), 256);
    L.clk_off = L.red_off + 256;  // step clock of the captured k-step graph
    L.total = L.clk_off + 256;
    return L;
}

bool side_bounded(int k) { return k != LB_BC_PERIODIC; }

lb_status validate(const lb_params *p) {
    if (!p) return fail(LB_EINVAL, "null parameters");
    if (p->nx < 1 || p->ny < 1) return fail(LB_EINVAL, "nx and ny must be >= 1");
    {
        const double plane = (double)align_up((size_t)p->nx, 64) * p->ny * (p->storage == LB_STORE_F32 ? 4.0 : 2.0) +
                             kPlanePadBytes;
        if (9.0 * plane >= 4294967296.0) return fail(LB_EINVAL, "grid too large (9 planes must span < 4 GiB)");
    }
    if (p->storage < 0 || p->storage > 2) return fail(LB_EINVAL, "storage");
    if (p->energy < 0 || p->energy > 1) return fail(LB_EINVAL, "energy");
    if (p->collision < 0 || p->collision > 1) return fail(LB_EINVAL, "collision");
    if (p->visc < 0 || p->visc > 3) return fail(LB_EINVAL, "visc");
    if (p->rho_extrap < 0 || p->rho_extrap > 1) return fail(LB_EINVAL, "rho_extrap");
    if (!(p->rho0 > 0) || !(p->T0 > 0) || !(p->b > 0) || !(p->Pr > 0))
        return fail(LB_EINVAL, "rho0, T0, b and Pr must be positive");
    if (!(std::fabs(3.0 * p->R * p->T0 - 1.0) <= 1e-12)) return fail(LB_EINVAL, "lattice units need R*T0 = 1/3 (c = 1)");
    if (p->energy == LB_ENERGY_INTERNAL && p->heating)
        return fail(LB_EINVAL, "the heating term belongs to the total-energy form");
    if (p->visc == LB_VISC_CONST_TAU) {
        if (!(p->tau_f > 0.5)) return fail(LB_EINVAL, "tau_f must exceed 1/2");
    } else if (!(p->mu_ref > 0) || !(p->T_ref > 0)) {
        return fail(LB_EINVAL, "mu_ref and T_ref must be positive");
    }
    if (p->visc == LB_VISC_SUTHERLAND && !(p->suth_S >= 0)) return fail(LB_EINVAL, "suth_S must be >= 0");
    if (p->s_e > 0 && !(p->s_e < 2)) return fail(LB_EINVAL, "s_e must lie in (0, 2)");
    if (p->s_zeta > 0 && !(p->s_zeta < 2)) return fail(LB_EINVAL, "s_zeta must lie in (0, 2)");
    if (!(p->s_q > 0 && p->s_q < 2)) return fail(LB_EINVAL, "s_q must lie in (0, 2)");
    if (!(p->tau_rho > 0.5) || !(p->tau_j > 0.5)) return fail(LB_EINVAL, "tau_rho and tau_j must exceed 1/2");
    if (!std::isfinite(p->g)) return fail(LB_EINVAL, "g");
    const int *k = nullptr;
    int kinds[4];
    for (int s = 0; s < 4; ++s) {
        kinds[s] = p->side[s].kind;
        if (kinds[s] < 0 || kinds[s] > 4) return fail(LB_EINVAL, "side kind");
    }
    (void)k;
    if (side_bounded(kinds[0]) != side_bounded(kinds[1]) || side_bounded(kinds[2]) != side_bounded(kinds[3]))
        return fail(LB_EINVAL, "both sides of an axis must be periodic or both bounded");
    for (int s = 0; s < 4; ++s) {
        if (kinds[s] == LB_BC_INLET && s != 0) return fail(LB_EINVAL, "inlet only at x-");
        if (kinds[s] == LB_BC_OUTLET && s != 1) return fail(LB_EINVAL, "outlet only at x+");
    }
    const bool io = kinds[0] == LB_BC_INLET || kinds[1] == LB_BC_OUTLET || kinds[1] == LB_BC_INLET ||
                    kinds[0] == LB_BC_OUTLET;
    if (io && side_bounded(kinds[2])) return fail(LB_EINVAL, "inlet/outlet need a periodic y axis");
    if ((side_bounded(kinds[0]) && p->nx < 3) || (side_bounded(kinds[2]) && p->ny < 3))
        return fail(LB_EINVAL, "a bounded axis needs at least 3 nodes");
    if (((kinds[0] == LB_BC_ADIABATIC || kinds[1] == LB_BC_ADIABATIC) && p->nx < 4) ||
        ((kinds[2] == LB_BC_ADIABATIC || kinds[3] == LB_BC_ADIABATIC) && p->ny < 4))
        return fail(LB_EINVAL, "an axis with an adiabatic wall needs at least 4 nodes");
    const double cs = 1.0 / std::sqrt(3.0);
    for (int s = 0; s < 4; ++s) {
        const lb_side &sd = p->side[s];
        if (kinds[s] == LB_BC_WALL || kinds[s] == LB_BC_ADIABATIC) {
            if (!(std::hypot(sd.ux, sd.uy) < cs)) return fail(LB_EINVAL, "wall speed must stay below c_s");
            if (kinds[s] == LB_BC_WALL && !(sd.T > 0)) return fail(LB_EINVAL, "wall temperature must be positive");
        }
        if (kinds[s] == LB_BC_INLET && (!(sd.period > 0) || !std::isfinite(sd.amp)))
            return fail(LB_EINVAL, "inlet needs period > 0 and a finite amplitude");
    }
    return LB_OK;
}

}  // namespace

struct lb_handle {
    lb_params p;
    Layout L;
    KArgs a;
    char *base;
    char *pops[2];
    float *snap;
    double *partials, *red;
    int cur;
    long n;
    int have_snap;
    hipStream_t stream;
    int strip_user;
    int bc;
    int walls;  // a side with a wall (Dirichlet or adiabatic)
    int red_blocks;
    double E0;
    int device;                      // HIP device current at lb_create
    long long *clk;                  // device step clock read by the graph's launches
    int graph_steps;                 // launches per captured graph (even), 0: host launches only
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // graphs starting from buffer 0 / 1
    hipGraph_t graph[2] = {nullptr, nullptr};
};

namespace {

void drop_graphs(lb_handle *h) {
    for (int c = 0; c < 2; ++c) {
        if (h->gexec[c]) (void)hipGraphExecDestroy(h->gexec[c]);
        if (h->graph[c]) (void)hipGraphDestroy(h->graph[c]);
        h->gexec[c] = nullptr;
        h->graph[c] = nullptr;
    }
}

void set_strip(lb_handle *h) {
    KArgs &a = h->a;
    a.tiles_x = (a.nx + kTile - 1) / kTile;
    int R = h->strip_user;
    if (R <= 0) {
        // 8-row strips for FP32 storage, 16 for the 16-bit codecs and for
        // FP32 grids with walls, whose FP64 row finishes make the two halo
        // rows of a strip dearer (measured best on 8192^2, 4096^2 and 2048^2;
        // the 2048^2 cavity in FP32: 156.6 us per step with 16 rows, 164.5
        // with 8); shorter ones, down to 1 row, while the grid would give
        // fewer wavefronts than a floor: 4096 (16 per CU) for fully periodic
        // grids, 2048 for bounded ones, whose step is heavier (measured on
        // periodic 1024^2, the 512^2 cavity and the 2048 x 256 channel in
        // FP32 and FP16)
        const bool f32 = h->p.storage == LB_STORE_F32;
        const int lw = f32 ? kLock<LB_STORE_F32> : kLock<LB_STORE_F16>;
        const long long bcols = (a.tiles_x + lw - 1) / lw;
        const long long floor_waves = (a.per_x && a.per_y) ? 4096 : 2048;
#ifdef LB_ARITH_FP64
        // FP64 arithmetic holds 256 VGPRs (2 wavefronts per SIMD): shorter and
        // more strips (measured on 8192^2: 2 rows 23.6 GLUPS, 8 rows 20.3)
        R = 2;
#else
        R = (f32 && !h->walls) ? 8 : 16;
#endif
        while (R > 1 && bcols * lw * ((a.ny + R - 1) / R) < floor_waves) R >>= 1;
    }
    a.strip_rows = R;
    a.n_strips = (a.ny + R - 1) / R;
    drop_graphs(h);
}

KArgs make_args(const lb_params *p, const Layout &L, double &E0out) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = p->nx;
    a.ny = p->ny;
    a.pitch = L.pitch;
    a.per_x = !side_bounded(p->side[0].kind);
    a.per_y = !side_bounded(p->side[2].kind);
    a.plane_bytes = (long long)L.plane_bytes;
    a.rs = 9 * L.pitch;
    a.pstride = (unsigned)(L.pitch * L.ssize);
    a.total = p->energy == LB_ENERGY_TOTAL;
    a.heat = a.total && p->heating;
    a.coupled = p->coupled != 0;
    a.corr = p->correction && p->coupled;
    a.bgk = p->collision == LB_COLLIDE_BGK;
    a.visc = p->visc;
    a.rho_press = p->rho_extrap == LB_RHO_PRESSURE;
    a.has_force = p->g != 0.0;
    // Dithered sums for the internal-energy form (the buoyancy-driven
    // cavities, run for hundreds of thousands of steps towards a steady
    // state).  Total-energy grids keep round-to-nearest: their test flows are
    // one-dimensional by symmetry (Couette, plane acoustic waves), which exact
    // rounding preserves column by column, and some of them (the mu ~ T
    // Couette at Ma = 0.35, the coupled acoustic wave at Pr = 5) are unstable
    // to transverse perturbations in the scheme itself (the FP64 reference
    // diverges too once seeded with 1e-10 of noise).
    a.dither = p->energy == LB_ENERGY_INTERNAL;
    const double E0 = 0.5 * p->b * p->R * p->T0;
    E0out = E0;
    a.rho0 = (real)p->rho0;
    a.E0 = (real)E0;
    a.inv_E0 = (real)(1.0 / E0);
    a.g = (real)p->g;
    a.half_g = (real)(0.5 * p->g);
    a.Pr = (real)p->Pr;
    if (p->visc == LB_VISC_CONST_TAU) {
        const double tau = p->tau_f, snu = 1.0 / tau;
        const double tau_h = (tau - 0.5) / p->Pr;
        const double wh = 2.0 / (2.0 * tau_h + 1.0);
        a.s_nu = (real)snu;
        a.omega_h = (real)wh;
        a.kcoup = (real)((1.0 - 0.5 * wh) * (p->Pr - 1.0) / tau);
        a.s_e = (real)(p->s_e > 0 ? p->s_e : snu);
        a.s_z = (real)(p->s_zeta > 0 ? p->s_zeta : snu);
    } else {
        a.s_e = (real)p->s_e;
        a.s_z = (real)p->s_zeta;
    }
    a.tie_e = !(p->s_e > 0);
    a.tie_z = !(p->s_zeta > 0);
    a.s_q = (real)p->s_q;
    a.s_rho = (real)(1.0 / p->tau_rho);
    a.s_j = (real)(1.0 / p->tau_j);
    a.mu3 = (real)(3.0 * p->mu_ref);
    a.cT = (real)(p->T0 / p->T_ref);
    a.visc_n = (real)p->visc_n;
    a.sT = (real)(p->suth_S / p->T_ref);
    for (int s = 0; s < 4; ++s) {
        a.side_kind[s] = p->side[s].kind;
        a.side_ux[s] = (real)p->side[s].ux;
        a.side_uy[s] = (real)p->side[s].uy;
        a.side_dth[s] = (real)(p->side[s].T / p->T0 - 1.0);
    }
    if (p->side[0].kind == LB_BC_INLET) {
        // Eq. 53-54: u = U0 s, rho = rho0 (1 + U0 s / c_s), T = T0 (1 + (gamma - 1) U0 s / c_s)
        const double gamma = (p->b + 2.0) / p->b;
        const double cs = std::sqrt(gamma * p->R * p->T0);
        const double U0 = p->side[0].amp;
        a.in_u = (real)U0;
        a.in_rho = (real)(p->rho0 * U0 / cs);
        a.in_th = (real)((gamma - 1.0) * U0 / cs);
        a.in_rate = 1.0 / p->side[0].period;
    }
    return a;
}

template <int ST, bool BC, class F>
void launch_step(lb_handle *h) {
    const KArgs &a = h->a;
    constexpr int LW = kLock<ST>;
    const int blocks = (a.tiles_x + LW - 1) / LW * a.n_strips;
    hipLaunchKernelGGL((k_step<ST, BC, F>), dim3(blocks), dim3(kWave * LW), 0, h->stream, a, h->pops[h->cur],
                       h->pops[1 - h->cur], (const long long *)nullptr, 0);
}

// Kernel and launch shape of one step, for graph capture.
template <int ST, bool BC, class F>
void step_kernel(const lb_handle *h, void *&fn, int &blocks, int &threads) {
    constexpr int LW = kLock<ST>;
    fn = (void *)k_step<ST, BC, F>;
    blocks = (h->a.tiles_x + LW - 1) / LW * h->a.n_strips;
    threads = kWave * LW;
}

typedef void (*step_fn)(lb_handle *);
typedef void (*kern_fn)(const lb_handle *, void *&, int &, int &);
// kind: 0 periodic with runtime switches, 1 bounded without walls (inlet,
// outlet), 2 periodic main configuration, 3 bounded with walls, 4 bounded
// with walls in the cavity configuration
kern_fn pick_kernel(int st, int kind) {
    static const kern_fn tbl[3][5] = {
        {step_kernel<LB_STORE_F32, false, Dyn>, step_kernel<LB_STORE_F32, true, Dyn>,
         step_kernel<LB_STORE_F32, false, Head>, step_kernel<LB_STORE_F32, true, DynW>,
         step_kernel<LB_STORE_F32, true, CavW>},
        {step_kernel<LB_STORE_F16, false, Dyn>, step_kernel<LB_STORE_F16, true, Dyn>,
         step_kernel<LB_STORE_F16, false, Head>, step_kernel<LB_STORE_F16, true, DynW>,
         step_kernel<LB_STORE_F16, true, CavW>},
        {step_kernel<LB_STORE_BF16, false, Dyn>, step_kernel<LB_STORE_BF16, true, Dyn>,
         step_kernel<LB_STORE_BF16, false, Head>, step_kernel<LB_STORE_BF16, true, DynW>,
         step_kernel<LB_STORE_BF16, true, CavW>},
    };
    return tbl[st][kind];
}

step_fn pick_step(int st, int kind) {
    static const step_fn tbl[3][5] = {
        {launch_step<LB_STORE_F32, false, Dyn>, launch_step<LB_STORE_F32, true, Dyn>,
         launch_step<LB_STORE_F32, false, Head>, launch_step<LB_STORE_F32, true, DynW>,
         launch_step<LB_STORE_F32, true, CavW>},
        {launch_step<LB_STORE_F16, false, Dyn>, launch_step<LB_STORE_F16, true, Dyn>,
         launch_step<LB_STORE_F16, false, Head>, launch_step<LB_STORE_F16, true, DynW>,
         launch_step<LB_STORE_F16, true, CavW>},
        {launch_step<LB_STORE_BF16, false, Dyn>, launch_step<LB_STORE_BF16, true, Dyn>,
         launch_step<LB_STORE_BF16, false, Head>, launch_step<LB_STORE_BF16, true, DynW>,
         launch_step<LB_STORE_BF16, true, CavW>},
    };
    return tbl[st][kind];
}

// the compile-time switch set Head applies
bool is_head(const KArgs &a) {
    return a.total && a.heat && a.coupled && a.corr && !a.has_force && !a.bgk && a.visc == LB_VISC_CONST_TAU;
}

// the compile-time switch set CavW applies (grids with walls only)
bool is_cavity(const KArgs &a) {
    return !a.total && !a.heat && a.coupled && a.corr && a.has_force && !a.bgk && a.visc != LB_VISC_CONST_TAU;
}

template <int ST, bool BC>
void launch_macros(lb_handle *h, float *o0, float *o1, float *o2, float *o3, int opitch, int full) {
    h->a.step = (unsigned)h->n;
    const int n = h->a.nx * h->a.ny;
    hipLaunchKernelGGL((k_macros<ST, BC>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, h->stream, h->a,
                       h->pops[h->cur], o0, o1, o2, o3, opitch, full, (float)h->p.T0);
}

template <int ST, bool BC>
void launch_pops(lb_handle *h, float *out, long long oplane, int q0, int nq) {
    h->a.step = (unsigned)h->n;
    const int n = h->a.nx * h->a.ny;
    hipLaunchKernelGGL((k_pops<ST, BC>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, h->stream, h->a,
                       h->pops[h->cur], out, oplane, q0, nq);
}

template <int ST, bool BC>
void launch_diag(lb_handle *h, int use_snap, int write_snap) {
    h->a.step = (unsigned)h->n;
    hipLaunchKernelGGL((k_diag<ST, BC>), dim3(h->red_blocks), dim3(kBlock), 0, h->stream, h->a, h->pops[h->cur],
                       h->snap, use_snap, write_snap, h->partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, h->stream, h->partials, h->red_blocks, h->red);
}

template <int ST, bool BC>
void launch_diag_to(lb_handle *h, int use_snap, int write_snap, double *out) {
    h->a.step = (unsigned)h->n;
    hipLaunchKernelGGL((k_diag<ST, BC>), dim3(h->red_blocks), dim3(kBlock), 0, h->stream, h->a, h->pops[h->cur],
                       h->snap, use_snap, write_snap, h->partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, h->stream, h->partials, h->red_blocks, out);
}

template <int ST, bool BC>
void launch_diag_partials(lb_handle *h, double *partials) {
    h->a.step = (unsigned)h->n;
    hipLaunchKernelGGL((k_diag<ST, BC>), dim3(h->red_blocks), dim3(kBlock), 0, h->stream, h->a, h->pops[h->cur],
                       h->snap, 0, 0, partials);
}

template <int ST>
void launch_init(lb_handle *h, const float *fields, long long fplane) {
    const int n = h->a.nx * h->a.ny;
    hipLaunchKernelGGL((k_init<ST>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, h->stream, h->a, fields,
                       fplane, h->pops[h->cur]);
}

#define DISPATCH(h, FN, ...)                                                                     \
    do {                                                                                         \
        const int st_ = (h)->p.storage, bc_ = (h)->bc;                                           \
        if (st_ == LB_STORE_F32) {                                                               \
            if (bc_) FN<LB_STORE_F32, true>(__VA_ARGS__); else FN<LB_STORE_F32, false>(__VA_ARGS__); \
        } else if (st_ == LB_STORE_F16) {                                                        \
            if (bc_) FN<LB_STORE_F16, true>(__VA_ARGS__); else FN<LB_STORE_F16, false>(__VA_ARGS__); \
        } else {                                                                                 \
            if (bc_) FN<LB_STORE_BF16, true>(__VA_ARGS__); else FN<LB_STORE_BF16, false>(__VA_ARGS__); \
        }                                                                                        \
    } while (0)

constexpr int kGraphSteps = 32;  // default launches per captured graph

// The k-step graph of a handle whose state starts in buffer c: k launches of
// the step kernel, launch i reading buffer (c + i) & 1 at time clk + i.  k is
// even, so a replay leaves the state in buffer c again.  The graph bakes the
// kernel arguments in; it is dropped whenever they change (strip height).
lb_status build_step_graph(lb_handle *h, int c, int kind) {
    void *fn = nullptr;
    int blocks = 0, threads = 0;
    pick_kernel(h->p.storage, kind)(h, fn, blocks, threads);
    HIPCHK(hipGraphCreate(&h->graph[c], 0));
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < h->graph_steps; ++i) {
        KArgs a = h->a;
        const char *src = h->pops[(c + i) & 1];
        char *dst = h->pops[(c + i + 1) & 1];
        const long long *clk = h->clk;
        int sub = i;
        void *args[5] = {(void *)&a, (void *)&src, (void *)&dst, (void *)&clk, (void *)&sub};
        hipKernelNodeParams kp{};
        kp.func = fn;
        kp.gridDim = dim3(blocks);
        kp.blockDim = dim3(threads);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, h->graph[c], prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
    }
    HIPCHK(hipGraphInstantiate(&h->gexec[c], h->graph[c], nullptr, nullptr, 0));
    return LB_OK;
}

lb_status run_diag(lb_handle *h, int use_snap, int write_snap, double out[kNred]) {
    DISPATCH(h, launch_diag, h, use_snap, write_snap);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, h->red, kNred * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

}  // namespace

// ------------------------------------------------- allocation-free entry point
// Partial sums of lb_diag_noalloc: kNred doubles per reduction block, at most
// kRedBlocks blocks (64 KiB).  Each GPU the library runs on holds its own copy
// until the process ends; every call on that GPU shares it.  Host code never
// uses this name as an address: it takes the device address of the current
// GPU's copy from hipGetSymbolAddress, once per device.
constexpr int kScratchDoubles = kRedBlocks * kNred;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on device dev (made current for the
// lookup, the caller's current device restored afterwards).
lb_status scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EINVAL, "device index beyond the 64 the library tracks");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess) return fail(LB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}
}  // namespace

extern "C" {

lb_status lb_validate(const lb_params *p) { return validate(p); }

size_t lb_state_bytes(const lb_params *p) {
    if (validate(p) != LB_OK) return 0;
    return layout_of(p).total;
}

lb_status lb_create(const lb_params *p, void *dev_state, size_t bytes, void *hip_stream, lb_handle **out) {
    if (!out) return fail(LB_EINVAL, "null output handle");
    *out = nullptr;
    lb_status s = validate(p);
    if (s != LB_OK) return s;
    const Layout L = layout_of(p);
    if (!dev_state) return fail(LB_EINVAL, "null device buffer");
    if (((uintptr_t)dev_state & 255) != 0) return fail(LB_EINVAL, "device buffer must be 256-byte aligned");
    if (bytes < L.total) return fail(LB_ENOMEM, "device buffer smaller than lb_state_bytes()");
    lb_handle *h = new lb_handle();
    h->p = *p;
    h->L = L;
    h->a = make_args(p, L, h->E0);
    h->base = (char *)dev_state;
    h->pops[0] = h->base;
    h->pops[1] = h->base + L.pops_bytes;
    h->snap = (float *)(h->base + L.snap_off);
    h->partials = (double *)(h->base + L.part_off);
    h->red = (double *)(h->base + L.red_off);
    h->clk = (long long *)(h->base + L.clk_off);
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    h->graph_steps = kGraphSteps;
    h->cur = 0;
    h->n = 0;
    h->have_snap = 0;
    h->stream = (hipStream_t)hip_stream;
    h->strip_user = 0;
    h->bc = !(h->a.per_x && h->a.per_y);
    h->walls = 0;
    for (int sd = 0; sd < 4; ++sd)
        if (p->side[sd].kind == LB_BC_WALL || p->side[sd].kind == LB_BC_ADIABATIC) h->walls = 1;
    const long long nodes = (long long)p->nx * p->ny;
    h->red_blocks = (int)std::min<long long>(kRedBlocks, (nodes + kBlock - 1) / kBlock);
    set_strip(h);
    *out = h;
    return LB_OK;
}

void lb_destroy(lb_handle *h) {
    if (!h) return;
    drop_graphs(h);
    delete h;
}

const char *lb_last_error(void) { return g_err.c_str(); }

long lb_time(const lb_handle *h) { return h ? h->n : -1; }

void *lb_stream(const lb_handle *h) { return h ? (void *)h->stream : nullptr; }

lb_status lb_set_strip_rows(lb_handle *h, int rows) {
    if (!h) return fail(LB_EINVAL, "null handle");
    if (rows < 0 || rows > 256 || (rows & (rows - 1)) != 0) return fail(LB_EINVAL, "strip rows: 0 or a power of two <= 256");
    h->strip_user = rows;
    set_strip(h);
    return LB_OK;
}

int lb_strip_rows(const lb_handle *h) { return h ? h->a.strip_rows : -1; }

lb_status lb_init(lb_handle *h, const double *rho, const double *ux, const double *uy, const double *T) {
    if (!h) return fail(LB_EINVAL, "null handle");
    const lb_params &p = h->p;
    const int pitch = h->L.pitch;
    const size_t fplane = (size_t)pitch * p.ny;
    std::vector<float> host(4 * fplane, 0.f);
    for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
            const size_t i = (size_t)y * p.nx + x, k = (size_t)y * pitch + x;
            host[k] = (float)(rho ? rho[i] - p.rho0 : 0.0);
            host[fplane + k] = (float)(ux ? ux[i] : 0.0);
            host[2 * fplane + k] = (float)(uy ? uy[i] : 0.0);
            host[3 * fplane + k] = (float)(T ? T[i] / p.T0 - 1.0 : 0.0);
        }
    h->cur = 0;
    h->n = 0;
    h->have_snap = 0;
    float *staging = (float *)h->pops[1];
    HIPCHK(hipMemcpyAsync(staging, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    switch (p.storage) {
    case LB_STORE_F32: launch_init<LB_STORE_F32>(h, staging, (long long)fplane); break;
    case LB_STORE_F16: launch_init<LB_STORE_F16>(h, staging, (long long)fplane); break;
    default: launch_init<LB_STORE_BF16>(h, staging, (long long)fplane); break;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb_step(lb_handle *h, long n) {
    if (!h) return fail(LB_EINVAL, "null handle");
    if (n < 0) return fail(LB_EINVAL, "negative step count");
    const int kind = h->bc ? (h->walls ? (is_cavity(h->a) ? 4 : 3) : 1) : (is_head(h->a) ? 2 : 0);
    // whole batches of graph_steps as replays of the captured graph, each
    // after a one-thread launch that sets the clock its launches read
    while (h->graph_steps > 0 && n >= h->graph_steps) {
        const int c = h->cur;
        if (!h->gexec[c]) {
            const lb_status st = build_step_graph(h, c, kind);
            if (st != LB_OK) {
                drop_graphs(h);
                return st;
            }
        }
        hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(1), 0, h->stream, h->clk, (long long)h->n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipGraphLaunch(h->gexec[c], h->stream));
        h->n += h->graph_steps;
        n -= h->graph_steps;
    }
    const step_fn fn = pick_step(h->p.storage, kind);
    for (long s = 0; s < n; ++s) {
        h->a.step = (unsigned)h->n;
        fn(h);
        h->cur ^= 1;
        h->n += 1;
    }
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_set_graph_steps(lb_handle *h, int k) {
    if (!h) return fail(LB_EINVAL, "null handle");
    if (k < 0 || k > 4096 || (k & 1)) return fail(LB_EINVAL, "graph steps: 0 or an even number <= 4096");
    h->graph_steps = k;
    drop_graphs(h);
    return LB_OK;
}

lb_status lb_macros(lb_handle *h, double *rho, double *ux, double *uy, double *T) {
    if (!h) return fail(LB_EINVAL, "null handle");
    const lb_params &p = h->p;
    const int pitch = h->L.pitch;
    const size_t fplane = (size_t)pitch * p.ny;
    float *st = (float *)h->pops[1 - h->cur];
    DISPATCH(h, launch_macros, h, st, st + fplane, st + 2 * fplane, st + 3 * fplane, pitch, 0);
    HIPCHK(hipGetLastError());
    std::vector<float> host(4 * fplane);
    HIPCHK(hipMemcpyAsync(host.data(), st, host.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
            const size_t i = (size_t)y * p.nx + x, k = (size_t)y * pitch + x;
            if (rho) rho[i] = p.rho0 + (double)host[k];
            if (ux) ux[i] = host[fplane + k];
            if (uy) uy[i] = host[2 * fplane + k];
            if (T) T[i] = p.T0 * (1.0 + (double)host[3 * fplane + k]);
        }
    return LB_OK;
}

lb_status lb_macros_device(lb_handle *h, float *rho, float *ux, float *uy, float *T) {
    if (!h) return fail(LB_EINVAL, "null handle");
    DISPATCH(h, launch_macros, h, rho, ux, uy, T, h->p.nx, 1);
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_populations(lb_handle *h, double *out) {
    if (!h || !out) return fail(LB_EINVAL, "null argument");
    const lb_params &p = h->p;
    const int pitch = h->L.pitch;
    const size_t fplane = (size_t)pitch * p.ny;
    float *st = (float *)h->pops[1 - h->cur];
    const int per_pass = (int)std::min<size_t>(18, h->L.pops_bytes / (fplane * sizeof(float)));
    // rest equilibria (rho0, 0, T0) in double
    const double w[9] = {4. / 9, 1. / 9, 1. / 9, 1. / 9, 1. / 9, 1. / 36, 1. / 36, 1. / 36, 1. / 36};
    const double e2[9] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    double rest[18];
    for (int q = 0; q < 9; ++q) {
        rest[q] = w[q] * p.rho0;
        rest[9 + q] = (p.energy == LB_ENERGY_TOTAL)
                          ? w[q] * (p.rho0 * h->E0 + 0.5 * p.rho0 * p.R * p.T0 * (3.0 * e2[q] - 2.0))
                          : w[q] * p.rho0 * h->E0;
    }
    std::vector<float> host((size_t)per_pass * fplane);
    for (int q0 = 0; q0 < 18; q0 += per_pass) {
        const int nq = std::min(per_pass, 18 - q0);
        DISPATCH(h, launch_pops, h, st, (long long)fplane, q0, nq);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(host.data(), st, (size_t)nq * fplane * sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int j = 0; j < nq; ++j)
            for (int y = 0; y < p.ny; ++y)
                for (int x = 0; x < p.nx; ++x)
                    out[((size_t)(q0 + j) * p.ny + y) * p.nx + x] =
                        rest[q0 + j] + (double)host[(size_t)j * fplane + (size_t)y * pitch + x];
    }
    return LB_OK;
}

lb_status lb_diag(lb_handle *h, double out[6]) {
    if (!h || !out) return fail(LB_EINVAL, "null argument");
    double r[kNred];
    lb_status s = run_diag(h, 0, 0, r);
    if (s != LB_OK) return s;
    const double N = (double)h->p.nx * h->p.ny;
    out[0] = N * h->p.rho0 + r[0];
    out[1] = N * h->p.rho0 * h->E0 + r[1];
    out[2] = r[2];
    out[3] = r[3];
    out[4] = r[4];
    out[5] = (double)h->n;
    if (r[4] > 0) return fail(LB_EUNSTABLE, "non-finite or non-positive moments on some nodes");
    return LB_OK;
}

lb_status lb_diag_noalloc(lb_handle *h, double *dev_out) {
    if (!h || !dev_out) return fail(LB_EINVAL, "null argument");
    if ((size_t)h->red_blocks * kNred > (size_t)kScratchDoubles)
        return fail(LB_EINVAL, "the reduction needs more partial sums than the static scratch holds (1024 blocks)");
    double *part = nullptr;
    const lb_status st = scratch_on(h->device, &part);
    if (st != LB_OK) return st;
    DISPATCH(h, launch_diag_partials, h, part);
    const double N = (double)h->p.nx * h->p.ny;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, h->stream, (const double *)part, h->red_blocks,
                       N * h->p.rho0, N * h->p.rho0 * h->E0, (double)h->n, dev_out);
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream) {
    if (!src || !dst) return fail(LB_EINVAL, "null argument");
    if ((bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(LB_EINVAL, "copy probe: 16-byte aligned pointers and a size in multiples of 16 bytes");
    const char *s = (const char *)src, *d = (const char *)dst;
    if (s < d + bytes && d < s + bytes) return fail(LB_EINVAL, "copy probe: overlapping buffers");
    if (bytes == 0) return LB_OK;
    const long long n = (long long)(bytes / 16);
    // up to 8192 blocks, each a contiguous chunk of whole rounds of the
    // block's lanes (kCopyUnroll vectors per lane per round)
    const long long round = (long long)kCopyUnroll * kBlock;
    const long long want = std::max<long long>(1, std::min<long long>(8192, (n + round - 1) / round));
    const long long chunk = ((n + want - 1) / want + round - 1) / round * round;
    const long long blocks = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)hip_stream, (const V4u *)src,
                       (V4u *)dst, n, chunk);
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_residual(lb_handle *h, int update, double *res) {
    if (!h || !res) return fail(LB_EINVAL, "null argument");
    double r[kNred];
    lb_status s = run_diag(h, h->have_snap, update ? 1 : 0, r);
    if (s != LB_OK) return s;
    *res = h->have_snap ? std::sqrt(r[5]) / std::sqrt(r[6]) : INFINITY;
    if (update) h->have_snap = 1;
    if (r[4] > 0) return fail(LB_EUNSTABLE, "non-finite or non-positive moments on some nodes");
    return LB_OK;
}

size_t lb_checkpoint_bytes(const lb_handle *h) {
    if (!h) return 0;
    return 64 + h->L.pops_bytes + h->L.snap_bytes;
}

lb_status lb_save(lb_handle *h, void *host_buf) {
    if (!h || !host_buf) return fail(LB_EINVAL, "null argument");
    char *b = (char *)host_buf;
    std::memset(b, 0, 64);
    const long long hdr[6] = {0x4C42444446ll, (long long)h->p.nx, (long long)h->p.ny, (long long)h->p.storage,
                              (long long)h->n, (long long)h->have_snap};
    std::memcpy(b, hdr, sizeof(hdr));
    HIPCHK(hipMemcpyAsync(b + 64, h->pops[h->cur], h->L.pops_bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(b + 64 + h->L.pops_bytes, h->snap, h->L.snap_bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb_load(lb_handle *h, const void *host_buf) {
    if (!h || !host_buf) return fail(LB_EINVAL, "null argument");
    const char *b = (const char *)host_buf;
    long long hdr[6];
    std::memcpy(hdr, b, sizeof(hdr));
    if (hdr[0] != 0x4C42444446ll || hdr[1] != h->p.nx || hdr[2] != h->p.ny || hdr[3] != h->p.storage)
        return fail(LB_EINVAL, "checkpoint does not match this grid");
    HIPCHK(hipMemcpyAsync(h->pops[0], b + 64, h->L.pops_bytes, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->snap, b + 64 + h->L.pops_bytes, h->L.snap_bytes, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->cur = 0;
    h->n = (long)hdr[4];
    h->have_snap = (int)hdr[5];
    return LB_OK;
}

}  // extern "C"

// =====================================================================
// Serving: continuous batching of many grids in one packed launch
// =====================================================================
struct lbs_server;

namespace {

constexpr int kMaxSlots = 512;
constexpr int kMaxItems = 1 << 18;
constexpr int kMultiBlocks = 2048;  // fixed grid of the packed step: 8192 wavefronts
// Strip height of the served grids, chosen per batch: 4 rows while the batch
// gives at least kServeWaves wavefronts at that height, else 2 (more, shorter
// items for a batch of small grids).  Measured on one MI355X: 16 requests of
// 64^2 and 128^2, 2.52 solves/s at 2 rows against 2.06 at 4 (FP16 2.93 against
// 2.14); 24 requests up to 256^2, 2.67 at 4 rows against 2.47 at 2; 8 rows
// slower on both.  The step's results do not depend on the strip height.
constexpr int kServeRowsLong = 4, kServeRowsShort = 2;
constexpr long kServeWaves = 2048;

// Work-list entries of one served grid per step with strips of `rows` rows:
// block items of kWavesPerBlock tiles for a wide grid (FP32 storage only),
// one per tile for a narrow one, times the strips.
int grid_is_wide(const lb_params *p) {
    return p->storage == LB_STORE_F32 && (p->nx + kTile - 1) / kTile >= kWavesPerBlock;
}
int work_items(const lb_params *p, int rows) {
    const int tiles = (p->nx + kTile - 1) / kTile;
    const int strips = (p->ny + rows - 1) / rows;
    return (grid_is_wide(p) ? (tiles + kWavesPerBlock - 1) / kWavesPerBlock : tiles) * strips;
}
// wavefronts of one step of a grid with strips of `rows` rows
long work_waves(const lb_params *p, int rows) {
    return (long)work_items(p, rows) * (grid_is_wide(p) ? kWavesPerBlock : 1);
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Plateau test of the convergence residual, applied once per check: the
// residual lies below 1e-2 of its largest value so far and has made no new
// minimum for max(10, checks / 2) checks, minima being counted from that
// maximum.  The flow's onset from a quiescent start makes the residual grow
// first, and the humps of a decaying transient stay well above its floor;
// true means the run has stalled at its rounding floor.
bool plateau_update(double r, double &peak, double &best, int &stall, int &checks) {
    ++checks;
    if (r > peak) {
        peak = best = r;
        stall = 0;
    } else if (r < best) {
        best = r;
        stall = 0;
    } else if (++stall >= std::max(10, checks / 2) && r < 1e-2 * peak) {
        return true;
    }
    return false;
}

struct Request {
    long id = 0;
    lb_params p{};
    std::vector<double> init;  // 4 fields [4][ny][nx], empty: rest state
    double tol = 0, best = INFINITY, peak = 0, residual = INFINITY;
    long max_steps = 0, steps = 0;
    int state = LBS_QUEUED, stall = 0, checks = 0, slot = -1;
    size_t off = 0, bytes = 0;
    int items = 0;  // work-list entries per step
    double t_submit = 0, t_admit = -1, t_done = -1;
    lb_handle *h = nullptr;
    std::vector<double> result;  // 4 fields once finished
};

}  // namespace

struct lbs_server {
    char *pool = nullptr;
    size_t pool_bytes = 0, hdr = 0;
    hipStream_t stream = nullptr;
    int storage = 0, k = 1;
    double t0 = 0;
    SlotDev *d_slots = nullptr;
    WorkItem *d_items = nullptr;
    int *d_nitems = nullptr;
    double *d_results = nullptr;
    std::vector<SlotDev> h_slots;
    std::vector<WorkItem> h_items;
    int h_counts[4] = {0, 0, 0, 0};  // wide and narrow items of part 0 (cavity grids), of part 1 (others)
    std::vector<double> h_results;
    std::vector<long> slot_req;               // slot -> request id or -1
    std::map<size_t, size_t> free_blocks;     // offset -> bytes
    std::map<long, Request> reqs;
    std::deque<long> queue;
    long next_id = 1;
    long items_resident = 0;  // work-list entries of the resident grids (short strips: the most)
    hipGraph_t graph[2] = {nullptr, nullptr};  // k-step batches of part 0 and part 1
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    double batches = 0, node_updates = 0, busy_s = 0, completed = 0;
};

namespace {

bool pool_alloc(lbs_server *S, size_t bytes, size_t &off) {
    bytes = align_up(bytes, 256);
    for (auto it = S->free_blocks.begin(); it != S->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            off = it->first;
            const size_t rest = it->second - bytes;
            S->free_blocks.erase(it);
            if (rest) S->free_blocks[off + bytes] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(lbs_server *S, size_t off, size_t bytes) {
    bytes = align_up(bytes, 256);
    auto it = S->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != S->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        S->free_blocks.erase(nx);
    }
    if (it != S->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            S->free_blocks.erase(it);
        }
    }
}

template <int ST>
void *multi_kernel(int part) {
    return part ? (void *)k_step_multi<ST, DynW> : (void *)k_step_multi<ST, CavW>;
}

// The k-step graph of one part of the work list: k launches of its packed
// kernel, launch i stepping every grid of the part from time n + i.
lb_status build_graph(lbs_server *S, int part) {
    HIPCHK(hipGraphCreate(&S->graph[part], 0));
    hipGraphNode_t prev = nullptr;
    void *fn = nullptr;
    switch (S->storage) {
    case LB_STORE_F32: fn = multi_kernel<LB_STORE_F32>(part); break;
    case LB_STORE_F16: fn = multi_kernel<LB_STORE_F16>(part); break;
    default: fn = multi_kernel<LB_STORE_BF16>(part); break;
    }
    for (int i = 0; i < S->k; ++i) {
        int ii = i, pp = part;
        const SlotDev *a0 = S->d_slots;
        const WorkItem *a1 = S->d_items;
        const int *a2 = S->d_nitems;
        void *args[5] = {(void *)&a0, (void *)&a1, (void *)&a2, (void *)&pp, (void *)&ii};
        hipKernelNodeParams kp{};
        kp.func = fn;
        kp.gridDim = dim3(kMultiBlocks);
        kp.blockDim = dim3(kBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, S->graph[part], prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
    }
    HIPCHK(hipGraphInstantiate(&S->exec[part], S->graph[part], nullptr, nullptr, 0));
    return LB_OK;
}

void drop_server_graphs(lbs_server *S) {
    for (int part = 0; part < 2; ++part) {
        if (S->exec[part]) (void)hipGraphExecDestroy(S->exec[part]);
        if (S->graph[part]) (void)hipGraphDestroy(S->graph[part]);
        S->exec[part] = nullptr;
        S->graph[part] = nullptr;
    }
}

lb_status admit(lbs_server *S) {
    while (!S->queue.empty()) {
        Request &r = S->reqs[S->queue.front()];
        int slot = -1;
        for (int i = 0; i < kMaxSlots; ++i)
            if (S->slot_req[i] < 0) {
                slot = i;
                break;
            }
        if (slot < 0) return LB_OK;
        // first in, first out: wait for room in the work list and the pool
        if (S->items_resident + r.items > kMaxItems) return LB_OK;
        size_t off;
        if (!pool_alloc(S, r.bytes, off)) return LB_OK;
        lb_handle *h = nullptr;
        lb_status st = lb_create(&r.p, S->pool + off, r.bytes, S->stream, &h);
        if (st != LB_OK) {
            pool_free(S, off, r.bytes);
            return st;
        }
        // the packed step gets its parallelism from many grids: long strips
        // (fewer halo rows per row computed) whatever the grid's size
        h->strip_user = kServeRowsLong;
        set_strip(h);
        const size_t N = (size_t)r.p.nx * r.p.ny;
        if (r.init.empty())
            st = lb_init(h, nullptr, nullptr, nullptr, nullptr);
        else
            st = lb_init(h, r.init.data(), r.init.data() + N, r.init.data() + 2 * N, r.init.data() + 3 * N);
        if (st != LB_OK) {
            lb_destroy(h);
            pool_free(S, off, r.bytes);
            return st;
        }
        // snapshot of the initial temperature, so that the first batch already
        // yields a residual (the same checks as a grid stepped on its own)
        DISPATCH(h, launch_diag_to, h, 0, 1, S->d_results + (size_t)slot * kNred);
        h->have_snap = 1;
        r.init.clear();
        r.init.shrink_to_fit();
        r.h = h;
        r.off = off;
        r.slot = slot;
        r.state = LBS_RUNNING;
        r.t_admit = now_s() - S->t0;
        S->items_resident += r.items;
        S->slot_req[slot] = r.id;
        S->queue.pop_front();
    }
    return LB_OK;
}

lb_status retire(lbs_server *S, Request &r, int state) {
    const size_t N = (size_t)r.p.nx * r.p.ny;
    r.result.assign(4 * N, 0.0);
    lb_status st = lb_macros(r.h, r.result.data(), r.result.data() + N, r.result.data() + 2 * N,
                             r.result.data() + 3 * N);
    r.state = state;
    r.t_done = now_s() - S->t0;
    S->slot_req[r.slot] = -1;
    r.slot = -1;
    lb_destroy(r.h);
    r.h = nullptr;
    pool_free(S, r.off, r.bytes);
    S->items_resident -= r.items;
    S->completed += 1;
    return st;
}

}  // namespace

extern "C" {

size_t lbs_pool_overhead(void) {
    return align_up(kMaxSlots * sizeof(SlotDev), 256) + align_up((size_t)kMaxItems * sizeof(WorkItem), 256) + 256 +
           align_up(kMaxSlots * kNred * sizeof(double), 256);
}

lb_status lbs_create(void *dev_pool, size_t pool_bytes, int storage, int k_steps, void *hip_stream, lbs_server **out) {
    if (!out) return fail(LB_EINVAL, "null output");
    *out = nullptr;
    if (!dev_pool || ((uintptr_t)dev_pool & 255)) return fail(LB_EINVAL, "pool must be a 256-byte aligned device buffer");
    if (storage < 0 || storage > 2) return fail(LB_EINVAL, "storage");
    if (k_steps < 1 || k_steps > 100000) return fail(LB_EINVAL, "k_steps must lie in 1..100000");
    const size_t hdr = lbs_pool_overhead();
    if (pool_bytes <= hdr) return fail(LB_ENOMEM, "pool smaller than the server tables");
    lbs_server *S = new lbs_server();
    S->pool = (char *)dev_pool;
    S->pool_bytes = pool_bytes;
    S->hdr = hdr;
    S->stream = (hipStream_t)hip_stream;
    S->storage = storage;
    S->k = k_steps;
    S->t0 = now_s();
    char *p = S->pool;
    S->d_slots = (SlotDev *)p;
    p += align_up(kMaxSlots * sizeof(SlotDev), 256);
    S->d_items = (WorkItem *)p;
    p += align_up((size_t)kMaxItems * sizeof(WorkItem), 256);
    S->d_nitems = (int *)p;
    p += 256;
    S->d_results = (double *)p;
    S->h_slots.resize(kMaxSlots);
    S->h_results.assign((size_t)kMaxSlots * kNred, 0.0);
    S->slot_req.assign(kMaxSlots, -1);
    S->free_blocks[hdr] = (pool_bytes - hdr) / 256 * 256;
    lb_status st = build_graph(S, 0);
    if (st == LB_OK) st = build_graph(S, 1);
    if (st != LB_OK) {
        drop_server_graphs(S);
        delete S;
        return st;
    }
    *out = S;
    return LB_OK;
}

lb_status lbs_submit(lbs_server *S, const lb_params *p, const double *rho, const double *ux, const double *uy,
                     const double *T, double tol, long max_steps, long *id) {
    if (!S || !p || !id) return fail(LB_EINVAL, "null argument");
    lb_status st = validate(p);
    if (st != LB_OK) return st;
    if (p->storage != S->storage) return fail(LB_EINVAL, "request storage differs from the server's");
    if (p->side[0].kind == LB_BC_INLET)
        return fail(LB_EINVAL, "the packed step serves grids without an inlet (walls, outlet or periodic sides)");
    if (max_steps < 1) return fail(LB_EINVAL, "max_steps must be >= 1");
    const Layout L = layout_of(p);
    if (L.total > S->pool_bytes - S->hdr) return fail(LB_ENOMEM, "request larger than the pool");
    if (work_items(p, kServeRowsShort) > kMaxItems) return fail(LB_EINVAL, "grid too large for the server's work list");
    Request r;
    r.id = S->next_id++;
    r.p = *p;
    r.tol = tol;
    r.max_steps = max_steps;
    r.bytes = L.total;
    r.items = work_items(p, kServeRowsShort);
    r.t_submit = now_s() - S->t0;
    if (rho || ux || uy || T) {
        const size_t N = (size_t)p->nx * p->ny;
        r.init.resize(4 * N);
        for (size_t i = 0; i < N; ++i) {
            r.init[i] = rho ? rho[i] : p->rho0;
            r.init[N + i] = ux ? ux[i] : 0.0;
            r.init[2 * N + i] = uy ? uy[i] : 0.0;
            r.init[3 * N + i] = T ? T[i] : p->T0;
        }
    }
    S->reqs[r.id] = std::move(r);
    S->queue.push_back(S->next_id - 1);
    *id = S->next_id - 1;
    return LB_OK;
}

lb_status lbs_advance(lbs_server *S, int *n_resident, int *n_queued) {
    if (!S) return fail(LB_EINVAL, "null server");
    lb_status st = admit(S);
    if (st != LB_OK) return st;
    // work list of every resident grid: the block items of the wide grids,
    // then the wavefront items of the narrow ones
    S->h_items.clear();
    std::vector<int> live;
    for (int slot = 0; slot < kMaxSlots; ++slot) {
        if (S->slot_req[slot] < 0) continue;
        Request &r = S->reqs[S->slot_req[slot]];
        lb_handle *h = r.h;
        SlotDev &sd = S->h_slots[slot];
        sd.a = h->a;
        sd.pops[0] = h->pops[0];
        sd.pops[1] = h->pops[1];
        sd.cur = h->cur;
        sd.n = h->n;
        live.push_back(slot);
    }
    // the batch's strip height (see kServeWaves)
    long waves = 0;
    for (int slot : live) waves += work_waves(&S->reqs[S->slot_req[slot]].p, kServeRowsLong);
    const int rows = waves >= kServeWaves ? kServeRowsLong : kServeRowsShort;
    for (int slot : live) {
        lb_handle *h = S->reqs[S->slot_req[slot]].h;
        if (h->a.strip_rows != rows) {
            h->strip_user = rows;
            set_strip(h);
        }
        S->h_slots[slot].a = h->a;
    }
    // part 0: the grids in the cavity configuration, part 1: the others;
    // within each, the wide grids' block items, then the narrow ones'
    for (int part = 0; part < 2; ++part) {
        for (int pass = 0; pass < 2; ++pass) {
            const size_t before = S->h_items.size();
            for (int slot : live) {
                const Request &r = S->reqs[S->slot_req[slot]];
                const KArgs &a = r.h->a;
                if (is_cavity(a) != (part == 0)) continue;
                const int wide = grid_is_wide(&r.p);
                if (wide != (pass == 0)) continue;
                const int step = wide ? kWavesPerBlock : 1;
                for (int sy = 0; sy < a.n_strips; ++sy)
                    for (int tx = 0; tx < a.tiles_x; tx += step) S->h_items.push_back(WorkItem{slot, tx, sy, 0});
            }
            S->h_counts[2 * part + pass] = (int)(S->h_items.size() - before);
        }
    }
    if (n_resident) *n_resident = (int)live.size();
    if (n_queued) *n_queued = (int)S->queue.size();
    if (live.empty()) return LB_OK;
    // admission keeps the list within kMaxItems
    if ((long)S->h_items.size() > S->items_resident) return fail(LB_EINVAL, "work list out of step with admission");
    if ((int)S->h_items.size() > kMaxItems) return fail(LB_ENOMEM, "work list overflow");
    const double t_start = now_s();
    const int nitems = (int)S->h_items.size();
    HIPCHK(hipMemcpyAsync(S->d_slots, S->h_slots.data(), kMaxSlots * sizeof(SlotDev), hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(S->d_items, S->h_items.data(), nitems * sizeof(WorkItem), hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(S->d_nitems, S->h_counts, 4 * sizeof(int), hipMemcpyHostToDevice, S->stream));
    for (int part = 0; part < 2; ++part)
        if (S->h_counts[2 * part] + S->h_counts[2 * part + 1] > 0) HIPCHK(hipGraphLaunch(S->exec[part], S->stream));
    // advance the grids' clocks, then the FP64 residual of each grid in one read-back
    for (int slot : live) {
        Request &r = S->reqs[S->slot_req[slot]];
        lb_handle *h = r.h;
        h->cur ^= (S->k & 1);
        h->n += S->k;
        S->node_updates += (double)r.p.nx * r.p.ny * S->k;
        double *out = S->d_results + (size_t)slot * kNred;
        DISPATCH(h, launch_diag_to, h, h->have_snap, 1, out);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(S->h_results.data(), S->d_results, kMaxSlots * kNred * sizeof(double), hipMemcpyDeviceToHost,
                          S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    S->busy_s += now_s() - t_start;
    S->batches += 1;
    for (int slot : live) {
        Request &r = S->reqs[S->slot_req[slot]];
        lb_handle *h = r.h;
        const double *res = &S->h_results[(size_t)slot * kNred];
        r.residual = h->have_snap ? std::sqrt(res[5]) / std::sqrt(res[6]) : INFINITY;
        h->have_snap = 1;
        r.steps = h->n;
        int done = -1;
        if (res[4] > 0) {
            done = LBS_UNSTABLE;
        } else if (r.residual < r.tol) {
            done = LBS_CONVERGED;
        } else if (r.steps >= r.max_steps) {
            done = LBS_STEP_CAP;
        } else if (std::isfinite(r.residual) && plateau_update(r.residual, r.peak, r.best, r.stall, r.checks)) {
            done = LBS_PLATEAU;
        }
        if (done >= 0) {
            st = retire(S, r, done);
            if (st != LB_OK) return st;
        }
    }
    return admit(S);
}

lb_status lbs_poll(lbs_server *S, long id, int *state, long *steps, double *residual, double times[3]) {
    if (!S) return fail(LB_EINVAL, "null server");
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(LB_EINVAL, "unknown request id");
    const Request &r = it->second;
    if (state) *state = r.state;
    if (steps) *steps = r.steps;
    if (residual) *residual = r.residual;
    if (times) {
        times[0] = r.t_submit;
        times[1] = r.t_admit;
        times[2] = r.t_done;
    }
    return LB_OK;
}

lb_status lbs_result(lbs_server *S, long id, double *rho, double *ux, double *uy, double *T) {
    if (!S) return fail(LB_EINVAL, "null server");
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(LB_EINVAL, "unknown request id");
    const Request &r = it->second;
    if (r.result.empty()) return fail(LB_EBUSY, "request not finished");
    const size_t N = (size_t)r.p.nx * r.p.ny;
    if (rho) std::memcpy(rho, r.result.data(), N * sizeof(double));
    if (ux) std::memcpy(ux, r.result.data() + N, N * sizeof(double));
    if (uy) std::memcpy(uy, r.result.data() + 2 * N, N * sizeof(double));
    if (T) std::memcpy(T, r.result.data() + 3 * N, N * sizeof(double));
    return LB_OK;
}

lb_status lbs_release(lbs_server *S, long id) {
    if (!S) return fail(LB_EINVAL, "null server");
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(LB_EINVAL, "unknown request id");
    if (it->second.state == LBS_QUEUED || it->second.state == LBS_RUNNING)
        return fail(LB_EBUSY, "request still queued or running");
    S->reqs.erase(it);
    return LB_OK;
}

lb_status lbs_stats(lbs_server *S, double out[6]) {
    if (!S || !out) return fail(LB_EINVAL, "null argument");
    size_t free_b = 0;
    for (auto &b : S->free_blocks) free_b += b.second;
    out[0] = S->batches;
    out[1] = S->node_updates;
    out[2] = S->busy_s;
    out[3] = S->completed;
    out[4] = (double)free_b;
    out[5] = (double)S->queue.size();
    return LB_OK;
}

void lbs_destroy(lbs_server *S) {
    if (!S) return;
    for (auto &kv : S->reqs)
        if (kv.second.h) lb_destroy(kv.second.h);
    drop_server_graphs(S);
    delete S;
}

}  // extern "C"
