// kernels.hpp -- gfx950 kernels of one lattice-Boltzmann phase-field time step.
//
// Method: Cartalade, Younsi & Plapp (arXiv:1602.07483).  Phase field, Sec. 3.2
// and the collision stage of Sec. 3.4 (eq. Collision_Stage); supersaturation,
// Sec. 3.3 (eqs. Supersaturation_Bis, Def_Jtot, Def_S, Def_Qu, LBE_Eq_Transport,
// Feq_Transport); temperature, Sec. 3.1 (eqs. LBE_Eq_Temp, EqFunction_Tempr,
// Source_Tempr); anti-trapping current, Sec. 2 (eq. AntiTrapping_Current).
//
// GPU formulation (same arithmetic as the paper's collide-then-stream, arranged
// for HBM bandwidth):
//  * Pull form, two lattices.  Thread x gathers g_i^{n+1}(x) = g_j*(y) from the
//    source node y of the incoming link (y = x - e_i inside the domain, the
//    node itself after bounce-back, the mirror node after a symmetry wall) and
//    evaluates that source's collision on the fly.  The non-local population
//    g_i(y + e_i, t) of eq. (Collision_Stage) is then always the destination's
//    own old population g_i^n(x), so the two reads per link are one shifted
//    and one aligned load of the same array.  Writing g^{n+1}(x) for all i
//    at once also yields phi^{n+1}(x) = sum_i g_i^{n+1}(x) in the same kernel.
//  * Node terms (a_s, N, eta_phi, Q_phi for phi; J_tot, S, Q_U/zeta, Q_theta for
//    U/theta) are computed once per node for the tile plus a one-node halo
//    and kept in LDS as two 4-vectors; the stencil field (phi^n, resp.
//    phi^{n+1} with 1/zeta) is staged in LDS with a two-node halo.  A block
//    owns a TX x TY column of nodes and marches through a slab of z planes,
//    rolling three planes of each.
//  * Links that cannot cross a wall (every link of a tile away from the
//    walls) take a fast path: compile-time direction, a uniform base pointer
//    and a 32-bit node offset.  Links that cross a wall take the general path.
//  * Populations are stored as deviations from their rest equilibria
//    (w_i phi, (A_i + B_i q/zeta) U, w_i theta) and updated in increment form,
//    in FP32 (or FP16/BF16 storage with FP32 arithmetic, or FP64 for
//    verification): the fields then absorb one rounding per step instead of
//    one per population.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.hpp"

namespace lbpf {

// --------------------------------------------------------------------------
// Storage codecs.  Every storage type holds deviations from the rest
// equilibrium; the codec is only the conversion to the arithmetic type.
// --------------------------------------------------------------------------
template <class S> struct Codec;
template <> struct Codec<float> {
    __device__ static float dec(float s) { return s; }
    __device__ static float enc(float v) { return v; }
};
template <> struct Codec<double> {
    __device__ static double dec(double s) { return s; }
    __device__ static double enc(double v) { return v; }
};
template <> struct Codec<__half> {
    __device__ static float dec(__half s) { return __half2float(s); }
    __device__ static __half enc(float v) { return __float2half_rn(v); }
};
template <> struct Codec<__hip_bfloat16> {
    __device__ static float dec(__hip_bfloat16 s) { return __bfloat162float(s); }
    __device__ static __hip_bfloat16 enc(float v) { return __float2bfloat16(v); }
};

// Population stores are never re-read by the writing kernel: stream them.
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(__half* p, __half v) {
    __builtin_nontemporal_store(__half_as_ushort(v), reinterpret_cast<unsigned short*>(p));
}
__device__ __forceinline__ void st_nt(__hip_bfloat16* p, __hip_bfloat16 v) {
    unsigned short b;
    __builtin_memcpy(&b, &v, sizeof(b));
    __builtin_nontemporal_store(b, reinterpret_cast<unsigned short*>(p));
}

// Raw buffer access.  One resource spans all Q arrays of a field (used when
// they total less than 4 GiB): every link then reads at the thread's own
// byte offset plus a per-direction scalar offset, so no vector instruction is
// spent on addressing; offsets past the end read 0 and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// CP is the cache policy of the load: 0 normal, 2 non-temporal (the line is
// not re-read by any block, so it should not displace lines that are).
template <class S, int CP = 0>
__device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, CP));
    else if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, CP));
    else
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, CP));
}
// streaming (non-temporal) stores
__device__ __forceinline__ void buf_st(float x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)v, (int)s, 2);
}
__device__ __forceinline__ void buf_st(double x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)v, (int)s, 2);
}
__device__ __forceinline__ void buf_st(__half x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(x), r, (int)v, (int)s, 2);
}
__device__ __forceinline__ void buf_st(__hip_bfloat16 x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, (int)v, (int)s, 2);
}

// Prefetch registers hold populations in a raw form, decoded where used.
// BF16 values are kept as zero-extended 32-bit words and widened with one
// explicit shift: written as a plain shift, the compiler folds the widening
// into half-register loads whose partial writes force a wait after each load.
template <class S> struct Raw {
    using type = S;
    template <int CP = 0>
    __device__ static S ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) { return buf_ld<S, CP>(r, v, s); }
    __device__ static S ldg(const S* p) { return *p; }
    __device__ static auto dec(S x) { return Codec<S>::dec(x); }
};
template <> struct Raw<__hip_bfloat16> {
    using type = unsigned;
    template <int CP = 0>
    __device__ static unsigned ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, CP);
    }
    __device__ static unsigned ldg(const __hip_bfloat16* p) {
        return (unsigned)*reinterpret_cast<const unsigned short*>(p);
    }
    __device__ static float dec(unsigned x) {
        unsigned o;
        asm("v_lshlrev_b32 %0, 16, %1" : "=v"(o) : "v"(x));
        return __builtin_bit_cast(float, o);
    }
};

// The populations h_i and f_i of one direction and node are pulled from the
// same source, so k_ut stores them side by side: element e of the pair array
// holds (h, f) at 2e and 2e + 1.  Pair<S> loads and stores both with one
// instruction (4 bytes per lane for 16-bit storage, 8 for FP32, 16 for
// FP64) and splits them where they are used.
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
// The FP32 and FP64 pairs are float and double vectors: reinterpreting one
// element of an integer vector as a float (bit_cast of x.y) is compiled, with
// packed FP32 instructions off, into a read of element 0.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
template <class S> struct Pair;
template <> struct Pair<float> {
    using type = f32x2_t;
    template <int CP = 0>
    __device__ static type ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(type, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, CP));
    }
    __device__ static type ldg(const float* p) { return *reinterpret_cast<const type*>(p); }
    __device__ static float h(type x) { return x.x; }
    __device__ static float f(type x) { return x.y; }
    __device__ static type enc2(float h, float f) { return type{h, f}; }
    __device__ static void st(type x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, (int)v, (int)s, 2);
    }
    __device__ static void stg(type x, float* p) { __builtin_nontemporal_store(x, reinterpret_cast<type*>(p)); }
};
template <> struct Pair<double> {
    using type = f64x2_t;
    template <int CP = 0>
    __device__ static type ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(type, __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, CP));
    }
    __device__ static type ldg(const double* p) { return *reinterpret_cast<const type*>(p); }
    __device__ static double h(type x) { return x.x; }
    __device__ static double f(type x) { return x.y; }
    __device__ static type enc2(double h, double f) { return type{h, f}; }
    __device__ static void st(type x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, x), r, (int)v, (int)s, 2);
    }
    __device__ static void stg(type x, double* p) { __builtin_nontemporal_store(x, reinterpret_cast<type*>(p)); }
};
template <> struct Pair<__half> {
    using type = unsigned;
    template <int CP = 0>
    __device__ static type ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, CP);
    }
    __device__ static type ldg(const __half* p) { return *reinterpret_cast<const unsigned*>(p); }
    __device__ static float h(type x) { return __half2float(__ushort_as_half((unsigned short)(x & 0xffffu))); }
    __device__ static float f(type x) { return __half2float(__ushort_as_half((unsigned short)(x >> 16))); }
    // encoded and packed as a two-half vector: each conversion is fused with
    // the FMA before it, the second writing the upper half of the first
    // one's register (no shift and merge)
    __device__ static type enc2(float h, float f) {
        typedef _Float16 h16x2_t __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(type, h16x2_t{__builtin_bit_cast(_Float16, Codec<__half>::enc(h)),
                                                __builtin_bit_cast(_Float16, Codec<__half>::enc(f))});
    }
    __device__ static void st(type x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(x, r, (int)v, (int)s, 2);
    }
    __device__ static void stg(type x, __half* p) { __builtin_nontemporal_store(x, reinterpret_cast<unsigned*>(p)); }
};
template <> struct Pair<__hip_bfloat16> {
    using type = unsigned;
    template <int CP = 0>
    __device__ static type ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, CP);
    }
    __device__ static type ldg(const __hip_bfloat16* p) { return *reinterpret_cast<const unsigned*>(p); }
    __device__ static float h(type x) { return __builtin_bit_cast(float, x << 16); }
    __device__ static float f(type x) { return __builtin_bit_cast(float, x & 0xffff0000u); }
    // both rounded (to nearest even) and packed by one conversion of a pair
    __device__ static type enc2(float h, float f) {
        typedef __bf16 b16x2_t __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(type, __builtin_convertvector(f32x2_t{h, f}, b16x2_t));
    }
    __device__ static void st(type x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(x, r, (int)v, (int)s, 2);
    }
    __device__ static void stg(type x, __hip_bfloat16* p) {
        __builtin_nontemporal_store(x, reinterpret_cast<unsigned*>(p));
    }
};

// Reciprocal and reciprocal square root: the hardware instructions (about
// 1 ulp) in FP32, exact operations in the FP64 verification build.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }

template <class T> struct alignas(4 * sizeof(T) > 16 ? 16 : 4 * sizeof(T)) V4 { T x, y, z, w; };
template <class T> struct alignas(2 * sizeof(T)) V2 { T x, y; };

// --------------------------------------------------------------------------
// Kernel constants (precomputed on the host in FP64, converted to T)
// --------------------------------------------------------------------------
template <class T>
struct Coef {
    int nx, ny, nz;
    int px;            // row pitch of every device array: nx rounded up to 32 elements
    int symm;          // bit f set: face f (-x,+x,-y,+y,-z,+z) is a symmetry wall
    int zslab;         // z planes per block
    int nbx, nby, nbz; // tiles per axis
    int remap;         // 1: deal contiguous runs of tiles to each XCD
    long long np;      // elements between two population arrays
    int aniso;
    T eps, delta;
    T inv2dx;          // 1 / (2 dx)
    T smin;            // |grad phi|^2 below which the normal is undefined
    T eta_c;           // W0^2 dt / (e^2 tau0 dx^2)           (eq. LBE_RelaxationTime)
    T cphi_e2;         // dt W0^2 / (dx tau0 e^2)               (eq. Feq_Phase)
    T dt_tau0;         // dt / tau0
    T lambda, Mcinf;
    T k, D;
    T inv_dt, inv_dx2;
    T jat_c;           // W0 / (2 sqrt 2)                       (eq. AntiTrapping_Current)
    T omU, omT;        // 1/eta_U, 1/eta_theta (eqs. RelaxationTime_Concentration, ThermalDiffusivity)
    T etaU;            // eta_U
    T dt;
    T jcoef;           // omU dt / (e^2 dx)
    T jt;              // dt / (e^2 dx)
    T adv[3];          // v dt / (e^2 dx): advection-diffusion heat equilibrium (Sec. 3.1)
    const T* advf;     // NULL, or v dt / (e^2 dx) per node, [3][nodes], replacing adv
    int has_adv;       // v != 0 or a velocity field
};

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Block index remapped so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) receives one contiguous run of tiles: halo and non-local re-reads of
// neighbouring tiles then hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int total, int remap) {
    if (!remap || (total & 7) != 0) return b;
    return (b & 7) * (total >> 3) + (b >> 3);
}

// r(phi) = q(phi)/zeta(phi), the same expression wherever a deviation is
// encoded or decoded.
template <class T>
__device__ __forceinline__ T r_of(T f, T zA, T zB) {
    return T(0.5) * (T(1) - f) * frcp(zA - zB * f);
}

// Source of the incoming link i at node (x,y,z) for pull streaming, general
// path.  Returns the source node (sx,sy,sz), the source direction j and the
// sign flips (fx,fy,fz) with e_j = (fx ex, fy ey, fz ez).  Walls: half-way
// bounce-back for no-flux faces, specular reflection for symmetry faces; a
// link crossing any no-flux face bounces back.
struct Src {
    int sx, sy, sz, j, fx, fy, fz;
};

template <class L, int I>
__device__ __forceinline__ Src source(int x, int y, int z, int nx, int ny, int nz, int symm) {
    constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
    Src s{x - ex, y - ey, z - ez, I, 1, 1, 1};
    int mask = 0;
    bool nf = false;
    if (ex != 0) {
        if (s.sx < 0) { mask |= 1; nf |= !(symm & 1); }
        else if (s.sx >= nx) { mask |= 1; nf |= !(symm & 2); }
    }
    if (ey != 0) {
        if (s.sy < 0) { mask |= 2; nf |= !(symm & 4); }
        else if (s.sy >= ny) { mask |= 2; nf |= !(symm & 8); }
    }
    if (ez != 0) {
        if (s.sz < 0) { mask |= 4; nf |= !(symm & 16); }
        else if (s.sz >= nz) { mask |= 4; nf |= !(symm & 32); }
    }
    if (mask) {
        if (nf) {
            s.sx = x; s.sy = y; s.sz = z; s.fx = -1; s.fy = -1; s.fz = -1;
        } else {
            if (mask & 1) { s.sx = x; s.fx = -1; }
            if (mask & 2) { s.sy = y; s.fy = -1; }
            if (mask & 4) { s.sz = z; s.fz = -1; }
        }
        s.j = find_dir<L>(s.fx * ex, s.fy * ey, s.fz * ez);
    }
    return s;
}

// Index of the direction opposite to I.
template <class L, int I>
constexpr int opposite_dir() {
    for (int i = 0; i < L::Q; ++i)
        if (L::ex(i) == -L::ex(I) && L::ey(i) == -L::ey(I) && L::ez(i) == -L::ez(I)) return i;
    return -1;
}

// Does the incoming link I of a node with the given face flags cross a wall?
struct Faces {
    bool xl, xh, yl, yh, zl, zh;   // node lies on the -x, +x, -y, +y, -z, +z face
};
template <class L, int I>
__device__ __forceinline__ bool crosses(const Faces& f) {
    constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
    bool c = false;
    if (ex > 0) c |= f.xl;
    if (ex < 0) c |= f.xh;
    if (ey > 0) c |= f.yl;
    if (ey < 0) c |= f.yh;
    if (ez > 0) c |= f.zl;
    if (ez < 0) c |= f.zh;
    return c;
}

// A value the compiler must treat as changed here: keeps per-direction base
// pointers from being hoisted into (and spilled from) scalar registers.
template <class V>
__device__ __forceinline__ V opaque(V v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Per-lane counterpart of opaque(): keeps loop-invariant per-lane work (the
// wall sources of the edge links) inside the branch that needs it instead of
// hoisted out of the z-march and spilled.
template <class V>
__device__ __forceinline__ V opaque_v(V v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Marks a loaded value as used on a path that has no use for it, so that its
// load is waited for there and not, later, by a write of the same register
// that would then also wait for every store issued since.
template <class V>
__device__ __forceinline__ void consume(const V& v) {
    asm volatile("" ::"v"(v));
}

// Compile-time loop over the directions.
template <int I, int Q>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, I>{});
        Unroll<I + 1, Q>::run(f);
    }
};
template <int Q>
struct Unroll<Q, Q> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

// --------------------------------------------------------------------------
// Anisotropy in unit-normal form.  With m = p/|p| (p = grad phi; a_s is even
// in n = -m), S4 = sum m^4:
//  cubic (eq. Anisotropic-Function_As): a = 1 - 3 eps + 4 eps S4,
//        |p| da/dp_a = 16 eps m_a (m_a^2 - S4);
//  K41/K61 (eq. As_K41-K61): a = 1 + eps (S4 - 3/5) + delta (3 S4 + 66 P - 17/7),
//        P = mx^2 my^2 mz^2,
//        |p| da/dp_a = 4 (eps + 3 delta) m_a (m_a^2 - S4)
//                      + 132 delta m_a m_b^2 m_c^2 (1 - 3 m_a^2).
// N = |p|^2 a da/dp (eq. TermesAnisotropes) = |p| a (|p| da/dp).
// --------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void aniso_terms(const Coef<T>& c, T px, T py, T pz, T& a, T& Nx, T& Ny,
                                            T& Nz) {
    const T s = px * px + py * py + pz * pz;
    if (!(s > c.smin)) {
        a = T(1); Nx = T(0); Ny = T(0); Nz = T(0);
        return;
    }
    const T inv = frsq(s);
    const T mag = s * inv;
    const T mx = px * inv, my = py * inv, mz = pz * inv;
    const T x2 = mx * mx, y2 = my * my, z2 = mz * mz;
    const T s4 = x2 * x2 + y2 * y2 + z2 * z2;
    T dx, dy, dz;
    if (c.aniso == 0) {
        a = T(1) - T(3) * c.eps + T(4) * c.eps * s4;
        const T f = T(16) * c.eps;
        dx = f * mx * (x2 - s4);
        dy = f * my * (y2 - s4);
        dz = f * mz * (z2 - s4);
    } else {
        a = T(1) + c.eps * (s4 - T(0.6)) + c.delta * (T(3) * s4 + T(66) * x2 * y2 * z2 - T(17.0 / 7.0));
        const T f = T(4) * (c.eps + T(3) * c.delta);
        const T g = T(132) * c.delta;
        dx = f * mx * (x2 - s4) + g * mx * y2 * z2 * (T(1) - T(3) * x2);
        dy = f * my * (y2 - s4) + g * my * x2 * z2 * (T(1) - T(3) * y2);
        dz = f * mz * (z2 - s4) + g * mz * x2 * y2 * (T(1) - T(3) * z2);
    }
    const T am = mag * a;
    Nx = am * dx; Ny = am * dy; Nz = am * dz;
}

// Boundary node (reading of "standard collision on boundary nodes", Sec. 3.4):
// the node lies on a no-flux face, i.e. one of its links crosses a no-flux wall.
__device__ __forceinline__ bool on_noflux_face(int x, int y, int z, int nx, int ny, int nz, int symm) {
    return (x == 0 && !(symm & 1)) || (x == nx - 1 && !(symm & 2)) ||
           (y == 0 && !(symm & 4)) || (y == ny - 1 && !(symm & 8)) ||
           (z == 0 && !(symm & 16)) || (z == nz - 1 && !(symm & 32));
}

// Shared per-block geometry of the 2.5D march.
template <int TX, int TY>
struct Tile {
    static constexpr int NT = TX * TY;
    static constexpr int PX = TX + 4, PY = TY + 4, PN = PX * PY;   // stencil field, halo 2
    static constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;   // node terms, halo 1
    int x0, y0, zs, ze, x, y, lt;
    bool active, xy_inner;
    Faces f;
    template <class T>
    __device__ Tile(const Coef<T>& c, int block) {
        const int total = c.nbx * c.nby * c.nbz;
        const int b = xcd_tile(block, total, c.remap);
        const int bx = b % c.nbx, by = (b / c.nbx) % c.nby, bz = b / (c.nbx * c.nby);
        x0 = bx * TX;
        y0 = by * TY;
        zs = bz * c.zslab;
        ze = min(zs + c.zslab, c.nz);
        const int ux = x0 + (int)threadIdx.x % TX, uy = y0 + (int)threadIdx.x / TX;
        lt = (uy - y0 + 1) * HX + (ux - x0 + 1);
        active = ux < c.nx && uy < c.ny;
        // a lane past the domain's last column or row works on the nearest
        // node of the tile and stores nothing
        x = min(ux, c.nx - 1);
        y = min(uy, c.ny - 1);
        // no node of the tile lies on an x or y face
        xy_inner = x0 > 0 && x0 + TX < c.nx && y0 > 0 && y0 + TY < c.ny;
        f.xl = x == 0; f.xh = x == c.nx - 1;
        f.yl = y == 0; f.yh = y == c.ny - 1;
        f.zl = false; f.zh = false;
    }
};

// The march.  Iteration zz of a block stages the stencil-field plane zz (A),
// computes the node terms of plane zz-1 (B) and pulls plane zz-2 (C).  All
// global loads an iteration needs (the field plane, the fields at the term
// nodes and the populations of the pulled plane) are issued together, before
// stage A: K_ut issues them at the end of the previous iteration and waits
// for them once; K_phi issues them at the top of the iteration and waits for
// each group where it is used.
// ==========================================================================
template <int TX, int TY>
struct March {
    using G = Tile<TX, TY>;
    static constexpr int NA = (G::PN + G::NT - 1) / G::NT;   // staged values per thread
    static constexpr int NB = (G::HN + G::NT - 1) / G::NT;   // term nodes per thread
};

// ==========================================================================
// K_phi: phase-field node terms, non-local collision and pull streaming.
// Reads g^n, phi^n, U^n, theta^n; writes g^{n+1}, phi^{n+1}.
//
// Stored: d_i = g_i - w_i phi (deviation from the rest equilibrium).  With
// the collision of eq. (Collision_Stage) at the source y of link i and the
// non-local value g_i^n(x):
//   g_i^{n+1}(x) = w_i phi_x + inc_i,
//   inc_i = w_i [A_y (phi_y - phi_x) + A_y Q_y dt/tau0 - e_j.(A_y V_y)]
//           + A_y (1 - omega_y) d_j(y) - (A_y - 1) d_i(x),
// A = 1/a_s^2 (1 on boundary nodes), V = omega c_phi N / e^2, so that
//   phi^{n+1}(x) = phi_x + sum_i inc_i,   d_i^{n+1}(x) = inc_i - w_i sum_i inc_i.
// Only small quantities are rounded besides the one update of phi.
// LDS terms: a = (A, A(1-omega), A Q dt/tau0, phi), b = (A V, 0).
// ==========================================================================
template <class L, class T, class S, int TX, int TY, bool BUF>
__device__ __forceinline__ void phi_body(const Coef<T>& c, int block, const S* __restrict__ gin,
                                         S* __restrict__ gout, const T* __restrict__ phin,
                                         const T* __restrict__ Un, const T* __restrict__ thn,
                                         T* __restrict__ phout) {
    using G = Tile<TX, TY>;
    using M = March<TX, TY>;
    __shared__ T sphi[3][G::PN];
    __shared__ V4<T> sta[3][G::HN];       // node terms, first 4-vector
    __shared__ V4<T> stb[3][G::HN];       // node terms, second 4-vector

    G tile(c, block);
    const int nx = c.nx, ny = c.ny, nz = c.nz, px = c.px;
    const unsigned plane = (unsigned)px * (unsigned)ny;
    const unsigned pbytes = (unsigned)((size_t)L::Q * (size_t)c.np * sizeof(S));
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(gin, BUF ? pbytes : 0u);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(gout, BUF ? pbytes : 0u);
    // The fields through buffer resources too: a lane's offset within a
    // plane is fixed for the whole march, the plane is a scalar offset.
    const unsigned fbytes = BUF ? (unsigned)((size_t)nz * plane * sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t rphi = make_rsrc(phin, fbytes), rU = make_rsrc(Un, fbytes),
                                 rth = make_rsrc(thn, fbytes);
    unsigned oa[M::NA], ob[M::NB];     // in-plane offsets of the staged and term nodes
#pragma unroll
    for (int k = 0; k < M::NA; ++k) {
        const int t = min((int)threadIdx.x + k * G::NT, G::PN - 1);
        oa[k] = (unsigned)(clampi(tile.y0 - 2 + t / G::PX, ny) * px + clampi(tile.x0 - 2 + t % G::PX, nx));
    }
#pragma unroll
    for (int k = 0; k < M::NB; ++k) {
        const int t = min((int)threadIdx.x + k * G::NT, G::HN - 1);
        ob[k] = (unsigned)(clampi(tile.y0 - 1 + t / G::HX, ny) * px + clampi(tile.x0 - 1 + t % G::HX, nx));
    }
    // In-plane byte offsets of the lane's node and its eight in-plane
    // neighbours, clamped to the domain.  The source of link i lies in plane
    // z - e_z at neighbour (-e_x, -e_y); clamping every coordinate gives a
    // link that crosses a wall an in-bounds stand-in, which stage C replaces.
    unsigned nbo[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
            nbo[dy][dx] = (unsigned)(clampi(tile.y + dy - 1, ny) * px + clampi(tile.x + dx - 1, nx)) *
                          (unsigned)sizeof(S);

    // registers filled at the top of each iteration
    T pa[M::NA];                       // phi^n of the staged plane
    T pu[M::NB], pt[M::NB];            // U^n, theta^n at the term nodes
    // d_j(source) and d_i(x) of the pulled plane, kept in the storage format
    // and decoded where used, so no conversion sits between the loads.
    typename Raw<S>::type pj[L::Q], pnl[L::Q];
    // The first four iterations of a slab fill the staged planes (stages A
    // and B only); every later one runs all three stages on the same loads
    // in the same order (lanes outside the domain read an in-bounds
    // stand-in).  With no path that skips a use, each group of loads is
    // waited for where it is used: the populations of stage C stay in flight
    // through stages A and B.
    auto prefetch = [&](int zz, auto full_c) {
        {   // A of iteration zz
            const size_t base = (size_t)clampi(zz, nz) * plane;
#pragma unroll
            for (int k = 0; k < M::NA; ++k) {
                if constexpr (BUF)
                    pa[k] = buf_ld<T>(rphi, oa[k] * (unsigned)sizeof(T), (unsigned)base * (unsigned)sizeof(T));
                else
                    pa[k] = phin[base + oa[k]];
            }
        }
        {   // B of iteration zz: terms of plane zz-1
            const size_t base = (size_t)clampi(zz - 1, nz) * plane;
#pragma unroll
            for (int k = 0; k < M::NB; ++k) {
                if constexpr (BUF) {
                    pu[k] = buf_ld<T>(rU, ob[k] * (unsigned)sizeof(T), (unsigned)base * (unsigned)sizeof(T));
                    pt[k] = buf_ld<T>(rth, ob[k] * (unsigned)sizeof(T), (unsigned)base * (unsigned)sizeof(T));
                } else {
                    pu[k] = Un[base + ob[k]];
                    pt[k] = thn[base + ob[k]];
                }
            }
        }
        if constexpr (decltype(full_c)::value) {   // C of iteration zz: plane zz-2
            const int z = zz - 2;
            const unsigned xi = (unsigned)z * plane + (unsigned)tile.y * px + tile.x;
            Faces f = tile.f;
            f.zl = z == 0;
            f.zh = z == nz - 1;
            const size_t np = (size_t)opaque(c.np);
            // planes z + 1, z, z - 1 (clamped), the source planes of e_z = -1, 0, 1
            const unsigned zo[3] = {(unsigned)clampi(z + 1, nz) * plane, (unsigned)z * plane,
                                    (unsigned)clampi(z - 1, nz) * plane};
            Unroll<0, L::Q>::run([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
                const int off = ex + ey * px + ez * (int)plane;
                if constexpr (BUF) {
                    pnl[I] = Raw<S>::template ld<>(rin, nbo[1][1], (unsigned)(I * np + zo[1]) * (unsigned)sizeof(S));
                    pj[I] = Raw<S>::template ld<>(rin, nbo[1 - ey][1 - ex],
                                                  (unsigned)(I * np + zo[1 + ez]) * (unsigned)sizeof(S));
                } else {
                    const bool cr = crosses<L, I>(f);    // wall links: read any in-bounds value
                    const S* gI = gin + (size_t)I * np;
                    const unsigned so = cr ? xi : xi - (unsigned)off;
                    pnl[I] = Raw<S>::ldg(gI + xi);
                    pj[I] = Raw<S>::ldg(gI + so);
                }
            });
        }
    };

    auto iteration = [&](int zz, auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        prefetch(zz, full_c);
        // A: stage phi^n plane zz
        {
            T* dst = sphi[(zz + 3) % 3];
#pragma unroll
            for (int k = 0; k < M::NA; ++k) {
                const int t = (int)threadIdx.x + k * G::NT;
                consume(pa[k]);
                if (t < G::PN) dst[t] = pa[k];
            }
        }
        __syncthreads();
        // B: node terms of plane zz-1 (needs phi^n planes zz-2 .. zz)
#pragma unroll
        for (int k = 0; k < M::NB; ++k) { consume(pu[k]); consume(pt[k]); }
        if (FULL || zz >= tile.zs) {
            const int pz = zz - 1;
            const T* fm = sphi[(pz + 2) % 3];
            const T* f0 = sphi[(pz + 3) % 3];
            const T* fp = sphi[(pz + 4) % 3];
            V4<T>* sa = sta[(pz + 3) % 3];
            V4<T>* sb = stb[(pz + 3) % 3];
#pragma unroll
            for (int k = 0; k < M::NB; ++k) {
                const int t = (int)threadIdx.x + k * G::NT;
                if (t >= G::HN) break;
                const int lx = t % G::HX, ly = t / G::HX;
                const int rx = tile.x0 - 1 + lx, ry = tile.y0 - 1 + ly;
                const int ctr = (ly + 1) * G::PX + (lx + 1);
                const T ph = f0[ctr];
                const T px = (f0[ctr + 1] - f0[ctr - 1]) * c.inv2dx;
                const T py = (f0[ctr + G::PX] - f0[ctr - G::PX]) * c.inv2dx;
                const T pzg = (fp[ctr] - fm[ctr]) * c.inv2dx;
                T a, Nx, Ny, Nz;
                aniso_terms(c, px, py, pzg, a, Nx, Ny, Nz);
                const T a2 = a * a;
                const T om = frcp(a2 * c.eta_c + T(0.5));            // eq. (LBE_RelaxationTime)
                const T one_m = T(1) - ph * ph;
                const T Qp = (ph - c.lambda * (c.Mcinf * pu[k] + pt[k]) * one_m) * one_m;  // eq. (LBE_SourceTerm)
                const bool bnd = on_noflux_face(rx, ry, pz, nx, ny, nz, c.symm);
                const T A = bnd ? T(1) : frcp(a2);
                const T av = A * om * c.cphi_e2;
                sa[t] = V4<T>{A, A * (T(1) - om), A * Qp * c.dt_tau0, ph};
                sb[t] = V4<T>{av * Nx, av * Ny, av * Nz, T(0)};
            }
        }
        __syncthreads();
        // C: pull plane zz-2 (terms of planes zz-3 .. zz-1 are ready).  Lanes
        // outside the domain compute a stand-in and store nothing.
        if constexpr (FULL) {
            const int z = zz - 2;
            const unsigned xi = (unsigned)z * plane + (unsigned)tile.y * px + tile.x;
            const int sl[3] = {(z + 2) % 3, (z + 3) % 3, (z + 4) % 3};   // planes z-1, z, z+1
            const T phx = sta[sl[1]][tile.lt].w;
            Faces f = tile.f;
            f.zl = z == 0;
            f.zh = z == nz - 1;
            const bool edge = !(tile.xy_inner && z > 0 && z < nz - 1);
            const size_t np = (size_t)opaque(c.np);
            T inc[L::Q];
            T dsum = T(0);
            // Every link as if its source x - e_i were inside the domain; on
            // edge tiles, a link that crosses a wall takes its source after
            // bounce-back or reflection instead (only the lanes it concerns).
            // When that source is the node itself (bounce-back, or reflection
            // across every face the link crosses), d_j(source) is the node's
            // own population of the opposite direction, already loaded as
            // d_i(x) of that direction; only other reflections load.
            auto wall_link = [&](auto ic) -> T {
                constexpr int I = decltype(ic)::value;
                constexpr int J = opposite_dir<L, I>();
                const Src s = source<L, I>(opaque_v(tile.x), opaque_v(tile.y), z, nx, ny, nz, c.symm);
                T dj;
                if (s.sx == tile.x && s.sy == tile.y && s.sz == z) {
                    dj = (T)Raw<S>::dec(pnl[J]);
                } else {
                    const size_t si = ((size_t)s.sz * ny + s.sy) * px + s.sx;
                    dj = (T)Codec<S>::dec(gin[(size_t)s.j * np + si]);
                }
                const T dnl = (T)Raw<S>::dec(pnl[I]);
                const int tsl = (s.sz + 3) % 3, tl = (s.sy - tile.y0 + 1) * G::HX + (s.sx - tile.x0 + 1);
                const V4<T> ta = sta[tsl][tl], tb = stb[tsl][tl];
                const T eAV = T(s.fx * L::ex(I)) * tb.x + T(s.fy * L::ey(I)) * tb.y +
                              T(s.fz * L::ez(I)) * tb.z;
                return T(L::w(I)) * (ta.x * (ta.w - phx) + ta.z - eAV) + ta.y * dj -
                       (ta.x - T(1)) * dnl;
            };
            auto fast = [&](auto ic, auto edge_c) {
                constexpr int I = decltype(ic)::value;
                constexpr bool EDGE = decltype(edge_c)::value;
                constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
                constexpr T wi = T(L::w(I));
                const int tl = tile.lt - ex - ey * G::HX;
                const V4<T> ta = sta[sl[1 - ez]][tl], tb = stb[sl[1 - ez]][tl];
                const T eAV = T(ex) * tb.x + T(ey) * tb.y + T(ez) * tb.z;
                T v = wi * (ta.x * (ta.w - phx) + ta.z - eAV) + ta.y * (T)Raw<S>::dec(pj[I]) -
                         (ta.x - T(1)) * (T)Raw<S>::dec(pnl[I]);
                if constexpr (EDGE && I != 0) {
                    consume(pj[I]);
                    consume(pnl[I]);
                    if (crosses<L, I>(f)) v = wall_link(ic);
                    __builtin_amdgcn_sched_barrier(0);   // one wall link at a time
                }
                inc[I] = v;
                dsum += v;
            };
            if (!edge)
                Unroll<0, L::Q>::run([&](auto ic) { fast(ic, std::false_type{}); });
            else
                Unroll<0, L::Q>::run([&](auto ic) { fast(ic, std::true_type{}); });
            // Both arms used every population; said once more where they
            // join, so that no load is taken as still in flight past it.
            Unroll<0, L::Q>::run([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                consume(pj[I]);
                consume(pnl[I]);
            });
            if (tile.active) {
                phout[xi] = phx + dsum;
                Unroll<0, L::Q>::run([&](auto ic) {
                    constexpr int I = decltype(ic)::value;
                    constexpr T wi = T(L::w(I));
                    const S v = Codec<S>::enc(inc[I] - wi * dsum);
                    if constexpr (BUF)
                        buf_st(v, rout, xi * (unsigned)sizeof(S), (unsigned)(I * np) * (unsigned)sizeof(S));
                    else
                        st_nt(&gout[(size_t)I * np + xi], v);
                });
            }
        }
    };
    int zz = tile.zs - 2;
    for (; zz < tile.zs + 2 && zz <= tile.ze + 1; ++zz) iteration(zz, std::false_type{});
    for (; zz <= tile.ze + 1; ++zz) iteration(zz, std::true_type{});
}

// ==========================================================================
// K_ut: supersaturation and heat node terms (with phi^{n+1}), BGK collisions
// and pull streaming.  Reads h^n, f^n, phi^n, phi^{n+1}, U^n, theta^n; writes
// h^{n+1}, f^{n+1}, U^{n+1}, theta^{n+1}.
//
// Stored deviations: dh_i = h_i - (A_i + B_i r^o) U with r^o = q/zeta of the
// phase field current when h was written (phi^n here), and df_i = f_i - w_i theta.
// With P = r^o U, C = omega_U (r - r^o) U (r from phi^{n+1}), S = source dt
// and K = omega_U dt J_tot / (e^2 dx) at the source y (eqs. LBE_Eq_Transport,
// Feq_Transport; A_0 = 1, B_0 = w_0 - 1, A_i = 0 and B_i = w_i otherwise):
//   h_i^{n+1}(x) = (A_i + B_i r^o_x) U_x + incU_i,
//   incU_i = [i>0] w_i (P_y - P_x) + B_i C_y + (1 - omega_U) dh_j(y) + w_i (S_y + e_j.K_y),
//   f_i^{n+1}(x) = w_i theta_x + incT_i,
//   incT_i = w_i (theta_y + (phi^{n+1}_y - phi^n_y)/2 - theta_x) + (1 - omega_theta) df_j(y)
//            [+ w_i e_j . A_y with the advection-diffusion equilibrium, A = omega_theta theta v dt/(e^2 dx)],
// then U^{n+1} = U_x + dU, theta^{n+1} = theta_x + dT and the new deviations
//   dh_i = incU_i - A_i dU + B_i [(r^o_x - r_x) U_x - r_x dU],  df_i = incT_i - w_i dT.
// For i > 0 the pull needs only Z = P + C + S, theta + dphi/2 and K of the
// source, so the halo terms in LDS are (Z, theta + dphi/2, Kx, Ky) and Kz;
// the tile's own (P, C, S, r) sit in a separate two-plane array.
// SU = false (pure substance, M c_inf = 0, where U does not act on phi):
// only theta is advanced; U is carried over unchanged and h is not touched.
// ST = false (isothermal, theta = 0 in the alloy benchmark of Sec. 4.2): only
// U is advanced; theta is carried over unchanged and f is not touched.
// ==========================================================================
template <class L, class T, class S, int TX, int TY, bool BUF, bool ADV = false, bool SU = true,
          bool ST = true>
__device__ __forceinline__ void ut_body(const Coef<T>& c, int block, const S* __restrict__ hin,
                                        S* __restrict__ hout, const S* __restrict__ fin,
                                        S* __restrict__ fout, const T* __restrict__ phio,
                                        const T* __restrict__ phnew, const T* __restrict__ Un,
                                        const T* __restrict__ thn, T* __restrict__ Uout,
                                        T* __restrict__ thout) {
    using G = Tile<TX, TY>;
    using M = March<TX, TY>;
    __shared__ V2<T> sphi[3][G::PN];      // (phi^{n+1}, 1/zeta)
    // Kz with halo; with advection also A = omega_theta theta v dt/(e^2 dx)
    using KT = std::conditional_t<ADV, V4<T>, T>;
    __shared__ V4<T> sta[3][G::HN];       // (Z, theta + dphi/2, Kx, Ky) with halo
    __shared__ KT stk[3][G::HN];
    __shared__ V4<T> sown[2][G::NT];      // (P, C, S, r) of the tile's own nodes

    G tile(c, block);
    const int nx = c.nx, ny = c.ny, nz = c.nz, px = c.px;
    const unsigned plane = (unsigned)px * (unsigned)ny;
    const T k = c.k;
    const T zA = T(0.5) * (T(1) + k), zB = T(0.5) * (T(1) - k);
    const T omU1 = T(1) - c.omU, omT1 = T(1) - c.omT;
    // With both fields solved, h and f sit side by side in one pair array
    // (Pair<S>), addressed through hin/hout.
    constexpr bool PAIR = SU && ST;
    constexpr unsigned PS = PAIR ? 2u * (unsigned)sizeof(S) : (unsigned)sizeof(S);   // bytes per element
    const unsigned pbytes = (unsigned)((size_t)L::Q * (size_t)c.np * PS);
    const __amdgpu_buffer_rsrc_t rhin = make_rsrc(hin, BUF ? pbytes : 0u);
    const __amdgpu_buffer_rsrc_t rfin = make_rsrc(fin, BUF ? pbytes : 0u);
    const __amdgpu_buffer_rsrc_t rhout = make_rsrc(hout, BUF ? pbytes : 0u);
    const __amdgpu_buffer_rsrc_t rfout = make_rsrc(fout, BUF ? pbytes : 0u);

    T pa[M::NA];                          // phi^{n+1} of the staged plane
    T po_[M::NB], pu[M::NB], pt[M::NB];   // phi^n, U^n, theta^n at the term nodes
    T pv[ADV ? 3 : 1][ADV ? M::NB : 1];   // advective velocity at the term nodes (field)
    [[maybe_unused]] const size_t nodes = (size_t)plane * (size_t)nz;
    // dh_j, df_j of the pulled plane's sources, raw: as pairs, or one array each
    typename Pair<S>::type pp_[PAIR ? L::Q : 1];
    typename Raw<S>::type ph_[PAIR ? 1 : L::Q], pf_[PAIR ? 1 : L::Q];
    T pUx = T(0), pthx = T(0);            // U^n, theta^n of the pulled node
    auto prefetch = [&](int zz) {
        {
            const size_t base = (size_t)clampi(zz, nz) * plane;
#pragma unroll
            for (int kk = 0; kk < M::NA; ++kk) {
                const int t = (int)threadIdx.x + kk * G::NT;
                if (t < G::PN) {
                    const int gx = clampi(tile.x0 - 2 + t % G::PX, nx), gy = clampi(tile.y0 - 2 + t / G::PX, ny);
                    pa[kk] = phnew[base + (size_t)gy * px + gx];
                }
            }
        }
        if (zz >= tile.zs) {
            const size_t base = (size_t)clampi(zz - 1, nz) * plane;
#pragma unroll
            for (int kk = 0; kk < M::NB; ++kk) {
                const int t = (int)threadIdx.x + kk * G::NT;
                if (t < G::HN) {
                    const int gx = clampi(tile.x0 - 1 + t % G::HX, nx), gy = clampi(tile.y0 - 1 + t / G::HX, ny);
                    const size_t gi = base + (size_t)gy * px + gx;
                    po_[kk] = phio[gi];
                    if constexpr (SU) pu[kk] = Un[gi];
                    if constexpr (ST) pt[kk] = thn[gi];
                    if constexpr (ADV) {
                        if (c.advf) {
                            pv[0][kk] = c.advf[gi];
                            pv[1][kk] = c.advf[nodes + gi];
                            pv[2][kk] = c.advf[2 * nodes + gi];
                        }
                    }
                }
            }
        }
        if (zz >= tile.zs + 2 && tile.active) {
            const int z = zz - 2;
            const unsigned xi = (unsigned)z * plane + (unsigned)tile.y * px + tile.x;
            Faces f = tile.f;
            f.zl = z == 0;
            f.zh = z == nz - 1;
            const size_t np = (size_t)opaque(c.np);
            pUx = Un[xi];
            pthx = thn[xi];
            // On edge tiles a link that crosses a wall loads the populations
            // its source gives after bounce-back or reflection (element
            // (j, source) of the wall rule) together with the others, so the
            // collision of stage C waits for no load of its own.
            const bool edge = !(tile.xy_inner && z > 0 && z < nz - 1);
            if (!edge) {
                Unroll<0, L::Q>::run([&](auto ic) {
                    constexpr int I = decltype(ic)::value;
                    constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
                    const int off = ex + ey * px + ez * (int)plane;
                    if constexpr (BUF) {
                        const unsigned vx = xi * PS;
                        const unsigned sj = (unsigned)(I * np) * PS - (unsigned)off * PS;
                        // The pull is a bijection: with e_x = 0 and rows of whole
                        // 128-byte lines, every line of a source row is read by
                        // this block alone, once.
                        constexpr int CP = ex == 0 && (TX * PS) % 128 == 0 ? 2 : 0;
                        if constexpr (PAIR) {
                            pp_[I] = Pair<S>::template ld<CP>(rhin, vx, sj);
                        } else {
                            if constexpr (SU) ph_[I] = Raw<S>::template ld<CP>(rhin, vx, sj);
                            if constexpr (ST) pf_[I] = Raw<S>::template ld<CP>(rfin, vx, sj);
                        }
                    } else {
                        const size_t so = (size_t)I * np + (xi - (unsigned)off);
                        if constexpr (PAIR) {
                            pp_[I] = Pair<S>::ldg(hin + 2 * so);
                        } else {
                            if constexpr (SU) ph_[I] = Raw<S>::ldg(hin + so);
                            if constexpr (ST) pf_[I] = Raw<S>::ldg(fin + so);
                        }
                    }
                });
            } else {
                Unroll<0, L::Q>::run([&](auto ic) {
                    constexpr int I = decltype(ic)::value;
                    constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
                    const int off = ex + ey * px + ez * (int)plane;
                    size_t src = (size_t)I * np + (xi - (unsigned)off);   // element of dh_j, df_j at the source
                    if (crosses<L, I>(f)) {
                        const Src w = source<L, I>(opaque_v(tile.x), opaque_v(tile.y), z, nx, ny, nz, c.symm);
                        src = (size_t)w.j * np + ((size_t)w.sz * ny + w.sy) * px + w.sx;
                    }
                    if constexpr (BUF) {
                        const unsigned ve = (unsigned)src * PS;
                        if constexpr (PAIR) {
                            pp_[I] = Pair<S>::template ld<>(rhin, ve, 0u);
                        } else {
                            if constexpr (SU) ph_[I] = Raw<S>::template ld<>(rhin, ve, 0u);
                            if constexpr (ST) pf_[I] = Raw<S>::template ld<>(rfin, ve, 0u);
                        }
                    } else {
                        if constexpr (PAIR) {
                            pp_[I] = Pair<S>::ldg(hin + 2 * src);
                        } else {
                            if constexpr (SU) ph_[I] = Raw<S>::ldg(hin + src);
                            if constexpr (ST) pf_[I] = Raw<S>::ldg(fin + src);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one direction's sources at a time
                });
            }
        }
    };

    prefetch(tile.zs - 2);
    for (int zz = tile.zs - 2; zz <= tile.ze + 1; ++zz) {
        {
            V2<T>* dst = sphi[(zz + 3) % 3];
#pragma unroll
            for (int kk = 0; kk < M::NA; ++kk) {
                const int t = (int)threadIdx.x + kk * G::NT;
                if (t < G::PN) dst[t] = V2<T>{pa[kk], frcp(zA - zB * pa[kk])};
            }
        }
        __syncthreads();
        if (zz >= tile.zs) {
            const int pz = zz - 1;
            const V2<T>* fm = sphi[(pz + 2) % 3];
            const V2<T>* f0 = sphi[(pz + 3) % 3];
            const V2<T>* fp = sphi[(pz + 4) % 3];
            V4<T>* sa = sta[(pz + 3) % 3];
            KT* sk = stk[(pz + 3) % 3];
            V4<T>* so = sown[pz & 1];
#pragma unroll
            for (int kk = 0; kk < M::NB; ++kk) {
                const int t = (int)threadIdx.x + kk * G::NT;
                if (t >= G::HN) break;
                const int lx = t % G::HX, ly = t / G::HX;
                const int ctr = (ly + 1) * G::PX + (lx + 1);
                // phi^{n+1} and 1/zeta at the node and its six neighbours (mirror ghosts)
                const V2<T> c0 = f0[ctr];
                const V2<T> nb[6] = {f0[ctr + 1], f0[ctr - 1], f0[ctr + G::PX], f0[ctr - G::PX],
                                     fp[ctr], fm[ctr]};
                const T p0 = c0.x, w0 = c0.y;
                const T q0 = T(0.5) * (T(1) - p0);       // q(phi)
                const T r0 = q0 * w0;                    // q/zeta
                T qn[6], rn[6];
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    qn[d] = T(0.5) * (T(1) - nb[d].x);
                    rn[d] = qn[d] * nb[d].y;
                }
                const T Gx = (rn[0] - rn[1]) * c.inv2dx, Gy = (rn[2] - rn[3]) * c.inv2dx,
                        Gz = (rn[4] - rn[5]) * c.inv2dx;
                const T Fx = (nb[0].y - nb[1].y) * c.inv2dx, Fy = (nb[2].y - nb[3].y) * c.inv2dx,
                        Fz = (nb[4].y - nb[5].y) * c.inv2dx;
                const T gx_ = (nb[0].x - nb[1].x) * c.inv2dx, gy_ = (nb[2].x - nb[3].x) * c.inv2dx,
                        gz_ = (nb[4].x - nb[5].x) * c.inv2dx;
                const T po = po_[kk], u = SU ? pu[kk] : T(0), th = ST ? pt[kk] : T(0);
                const T dphi = p0 - po;
                if constexpr (!SU) {   // theta terms only
                    sa[t] = V4<T>{T(0), th + T(0.5) * dphi, T(0), T(0)};
                    if constexpr (ADV) {
                        const T ot = c.omT * th;
                        const T ax = c.advf ? pv[0][kk] : c.adv[0], ay = c.advf ? pv[1][kk] : c.adv[1],
                                az = c.advf ? pv[2][kk] : c.adv[2];
                        sk[t] = V4<T>{T(0), ot * ax, ot * ay, ot * az};
                    } else {
                        sk[t] = T(0);
                    }
                    continue;
                }
                const T dtphi = dphi * c.inv_dt;
                const T cu = T(1) + (T(1) - k) * u;
                // anti-trapping current, eq. (AntiTrapping_Current)
                T jx = T(0), jy = T(0), jz = T(0);
                const T s2 = gx_ * gx_ + gy_ * gy_ + gz_ * gz_;
                if (s2 > c.smin) {
                    const T f = -c.jat_c * cu * dtphi * frsq(s2);
                    jx = f * gx_; jy = f * gy_; jz = f * gz_;
                }
                // compact div(q grad(1/zeta))
                T div = T(0);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    div += T(0.5) * (q0 + qn[2 * a]) * (nb[2 * a].y - w0) -
                           T(0.5) * (q0 + qn[2 * a + 1]) * (w0 - nb[2 * a + 1].y);
                div *= c.inv_dx2;
                // J_tot (eq. Def_Jtot), S (eq. Def_S), Q_U/zeta (eq. Def_Qu)
                const T Du = c.D * u;
                const T Jx = Du * (Gx + q0 * Fx) + jx * w0;
                const T Jy = Du * (Gy + q0 * Fy) + jy * w0;
                const T Jz = Du * (Gz + q0 * Fz) + jz * w0;
                const T Sflux = Du * div + jx * Fx + jy * Fy + jz * Fz;
                const T src = Sflux + cu * T(0.5) * dtphi * w0;
                const T ro = r_of(po, zA, zB);
                const T P = ro * u, C = c.omU * (r0 - ro) * u, Ssrc = src * c.dt;
                sa[t] = V4<T>{P + C + Ssrc, th + T(0.5) * dphi, c.jcoef * Jx, c.jcoef * Jy};
                if constexpr (ADV) {
                    const T ot = c.omT * th;
                    const T ax = c.advf ? pv[0][kk] : c.adv[0], ay = c.advf ? pv[1][kk] : c.adv[1],
                            az = c.advf ? pv[2][kk] : c.adv[2];
                    sk[t] = V4<T>{c.jcoef * Jz, ot * ax, ot * ay, ot * az};
                } else {
                    sk[t] = c.jcoef * Jz;
                }
                if (lx >= 1 && lx <= TX && ly >= 1 && ly <= TY)
                    so[(ly - 1) * TX + (lx - 1)] = V4<T>{P, C, Ssrc, r0};
            }
        }
        __syncthreads();
        if (zz >= tile.zs + 2 && tile.active) {
            const int z = zz - 2;
            const unsigned xi = (unsigned)z * plane + (unsigned)tile.y * px + tile.x;
            const int sl[3] = {(z + 2) % 3, (z + 3) % 3, (z + 4) % 3};
            const V4<T> own = sown[z & 1][threadIdx.x];
            const T Px = own.x, Cx = own.y, Sx = own.z, rx = own.w;
            const T Ux = pUx, thx = pthx;
            Faces f = tile.f;
            f.zl = z == 0;
            f.zh = z == nz - 1;
            const bool edge = !(tile.xy_inner && z > 0 && z < nz - 1);
            const size_t np = (size_t)opaque(c.np);
            T iu[L::Q], it[L::Q];
            T du = T(0), dth = T(0);
            // the prefetched dh_j, df_j of link I, decoded
            auto dh_of = [&](auto ic) -> T {
                constexpr int I = decltype(ic)::value;
                if constexpr (PAIR) return (T)Pair<S>::h(pp_[I]);
                else if constexpr (SU) return (T)Raw<S>::dec(ph_[I]);
                else return T(0);
            };
            auto df_of = [&](auto ic) -> T {
                constexpr int I = decltype(ic)::value;
                if constexpr (PAIR) return (T)Pair<S>::f(pp_[I]);
                else if constexpr (ST) return (T)Raw<S>::dec(pf_[I]);
                else return T(0);
            };
            // A link that crosses a wall: source after bounce-back or reflection.
            auto wall_link = [&](auto ic, T& vu, T& vt) {
                constexpr int I = decltype(ic)::value;
                const Src s = source<L, I>(opaque_v(tile.x), opaque_v(tile.y), z, nx, ny, nz, c.symm);
                // loaded with the others from the wall rule's source
                const T dh = dh_of(ic), df = df_of(ic);
                const int tsl = (s.sz + 3) % 3, tl = (s.sy - tile.y0 + 1) * G::HX + (s.sx - tile.x0 + 1);
                const V4<T> ta = sta[tsl][tl];
                constexpr T wi = T(L::w(I));
                const int ejx = s.fx * L::ex(I), ejy = s.fy * L::ey(I), ejz = s.fz * L::ez(I);
                T eK = T(ejx) * ta.z + T(ejy) * ta.w;
                T eA = T(0);
                if constexpr (ADV) {
                    const V4<T> kv = stk[tsl][tl];
                    eK += T(ejz) * kv.x;
                    eA = T(ejx) * kv.y + T(ejy) * kv.z + T(ejz) * kv.w;
                } else {
                    eK += T(ejz) * stk[tsl][tl];
                }
                // I > 0 here: A_I = 0, B_I = w_I
                if constexpr (SU) vu = wi * (ta.x - Px + eK) + omU1 * dh;
                if constexpr (ST) vt = wi * (ta.y - thx + eA) + omT1 * df;
            };
            auto fast = [&](auto ic, auto edge_c) {
                constexpr int I = decltype(ic)::value;
                constexpr bool EDGE = decltype(edge_c)::value;
                constexpr int ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
                constexpr T wi = T(L::w(I));
                const int tl = tile.lt - ex - ey * G::HX;
                const V4<T> ta = sta[sl[1 - ez]][tl];
                T vu = T(0), vt = T(0);
                T eA = T(0);
                if constexpr (I == 0) {
                    if constexpr (SU) vu = (wi - T(1)) * Cx + wi * Sx + omU1 * dh_of(ic);
                } else {
                    T eK = T(ex) * ta.z + T(ey) * ta.w;
                    if constexpr (ADV) {
                        const V4<T> kv = stk[sl[1 - ez]][tl];
                        if constexpr (ez != 0) eK += T(ez) * kv.x;
                        eA = T(ex) * kv.y + T(ey) * kv.z + T(ez) * kv.w;
                    } else {
                        if constexpr (ez != 0) eK += T(ez) * stk[sl[1 - ez]][tl];
                    }
                    if constexpr (SU) vu = wi * (ta.x - Px + eK) + omU1 * dh_of(ic);
                }
                if constexpr (ST) vt = wi * (ta.y - thx + eA) + omT1 * df_of(ic);
                if constexpr (EDGE && I != 0) {
                    if (crosses<L, I>(f)) wall_link(ic, vu, vt);
                    __builtin_amdgcn_sched_barrier(0);   // one wall link at a time
                }
                iu[I] = vu; it[I] = vt;
                du += vu; dth += vt;
            };
            if (!edge)
                Unroll<0, L::Q>::run([&](auto ic) { fast(ic, std::false_type{}); });
            else
                Unroll<0, L::Q>::run([&](auto ic) { fast(ic, std::true_type{}); });
            Uout[xi] = SU ? Ux + du : Ux;
            thout[xi] = ST ? thx + dth : thx;
            // (r^o_x - r_x) U_x - r_x dU, with (r^o_x - r_x) U_x = -C_x / omega_U
            const T hb = -Cx * c.etaU - rx * du;
            Unroll<0, L::Q>::run([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                constexpr T wi = T(L::w(I));
                constexpr T Bi = (I == 0) ? T(L::w(0)) - T(1) : wi;
                const T dhv = (I == 0) ? iu[I] - du + Bi * hb : iu[I] + Bi * hb;
                const T dfv = it[I] - wi * dth;
                const S hv = Codec<S>::enc(dhv), fv = Codec<S>::enc(dfv);
                if constexpr (BUF) {
                    const unsigned vx = xi * PS, sI = (unsigned)(I * np) * PS;
                    if constexpr (PAIR) {
                        Pair<S>::st(Pair<S>::enc2(dhv, dfv), rhout, vx, sI);
                    } else {
                        if constexpr (SU) buf_st(hv, rhout, vx, sI);
                        if constexpr (ST) buf_st(fv, rfout, vx, sI);
                    }
                } else {
                    if constexpr (PAIR) {
                        Pair<S>::stg(Pair<S>::enc2(dhv, dfv), hout + 2 * ((size_t)I * np + xi));
                    } else {
                        if constexpr (SU) st_nt(&hout[(size_t)I * np + xi], hv);
                        if constexpr (ST) st_nt(&fout[(size_t)I * np + xi], fv);
                    }
                }
            });
        }
        if (zz + 1 <= tile.ze + 1) prefetch(zz + 1);
    }
}

// --------------------------------------------------------------------------
// Launch forms.  Single domain: the constants travel as kernel arguments and
// block b is tile b.  Batch: every block reads its (domain, tile) from a work
// table and the domain's constants and buffers from a descriptor array; the
// populations and fields of parity par are read and those of 1-par written.
// --------------------------------------------------------------------------
template <class L, class T, class S, int TX, int TY, bool BUF>
__global__ __launch_bounds__(TX * TY, (sizeof(T) == 4 ? 4 : 1)) void k_phi(
    const Coef<T> c, const S* __restrict__ gin, S* __restrict__ gout, const T* __restrict__ phin,
    const T* __restrict__ Un, const T* __restrict__ thn, T* __restrict__ phout) {
    phi_body<L, T, S, TX, TY, BUF>(c, blockIdx.x, gin, gout, phin, Un, thn, phout);
}

template <class L, class T, class S, int TX, int TY, bool BUF, bool ADV = false, bool SU = true,
          bool ST = true>
__global__ __launch_bounds__(TX * TY, (sizeof(T) == 4 ? 3 : 1)) void k_ut(
    const Coef<T> c, const S* __restrict__ hin, S* __restrict__ hout, const S* __restrict__ fin,
    S* __restrict__ fout, const T* __restrict__ phio, const T* __restrict__ phnew,
    const T* __restrict__ Un, const T* __restrict__ thn, T* __restrict__ Uout, T* __restrict__ thout) {
    ut_body<L, T, S, TX, TY, BUF, ADV, SU, ST>(c, blockIdx.x, hin, hout, fin, fout, phio, phnew, Un, thn,
                                               Uout, thout);
}

template <class T>
struct DomainDesc {
    Coef<T> c[2];      // constants with the tiling of k_phi [0] and k_ut [1]
    void* pop[3][2];   // g, h, f populations per parity
    T* fld[3][2];      // phi, U, theta per parity
};

template <class L, class T, class S, int TX, int TY>
__global__ __launch_bounds__(TX * TY, (sizeof(T) == 4 ? 4 : 1)) void k_phi_batch(
    const DomainDesc<T>* __restrict__ dd, const int2* __restrict__ work, int par) {
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;   // padding entry: the whole block leaves
    // The descriptor is read once into registers, as the single-domain
    // kernel receives it as arguments: read through a reference, its fields
    // are re-loaded inside the march, and each scalar load's wait also
    // drains the LDS operations in flight.
    const int a = par, b = 1 - par;
    const Coef<T> c = dd[wk.x].c[0];
    const S* gin = (const S*)dd[wk.x].pop[0][a];
    S* gout = (S*)dd[wk.x].pop[0][b];
    const T *phin = dd[wk.x].fld[0][a], *Un = dd[wk.x].fld[1][a], *thn = dd[wk.x].fld[2][a];
    T* phout = dd[wk.x].fld[0][b];
    phi_body<L, T, S, TX, TY, true>(c, wk.y, gin, gout, phin, Un, thn, phout);
}

template <class L, class T, class S, int TX, int TY>
__global__ __launch_bounds__(TX * TY, (sizeof(T) == 4 ? 3 : 1)) void k_ut_batch(
    const DomainDesc<T>* __restrict__ dd, const int2* __restrict__ work, int par) {
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;   // padding entry: the whole block leaves
    const int a = par, b = 1 - par;
    const Coef<T> c = dd[wk.x].c[1];   // read once (see k_phi_batch)
    const S* hin = (const S*)dd[wk.x].pop[1][a];
    S* hout = (S*)dd[wk.x].pop[1][b];
    const S* fin = (const S*)dd[wk.x].pop[2][a];
    S* fout = (S*)dd[wk.x].pop[2][b];
    const T *phio = dd[wk.x].fld[0][a], *phnew = dd[wk.x].fld[0][b];
    const T *Un = dd[wk.x].fld[1][a], *thn = dd[wk.x].fld[2][a];
    T *Uout = dd[wk.x].fld[1][b], *thout = dd[wk.x].fld[2][b];
    ut_body<L, T, S, TX, TY, true>(c, wk.y, hin, hout, fin, fout, phio, phnew, Un, thn, Uout, thout);
}

// ==========================================================================
// Initial populations = equilibria of the given fields (plain per-node kernel,
// runs once), stored as deviations.  g: eq. (Feq_Phase) with N from grad phi,
// deviation -w_i e_i.N c_phi/e^2; h: eq. (Feq_Transport) with J_tot =
// D (grad(q/zeta) + q grad(1/zeta)) U (no anti-trapping current without a
// time derivative), deviation B_i e_i.J dt/(e^2 dx); f: eq. (EqFunction_Tempr),
// deviation 0.
// ==========================================================================
template <class L, class T, class S>
__global__ __launch_bounds__(256) void k_init(const Coef<T> c, S* __restrict__ g, S* __restrict__ h,
                                              S* __restrict__ f, int hs,   // element stride of h and f
                                              const T* __restrict__ phi,
                                              const T* __restrict__ U, const T* __restrict__ th,
                                              int parts) {   // bit 0: g, bit 1: h and f (on lattice L)
    const int nx = c.nx, ny = c.ny, nz = c.nz, px = c.px;
    const size_t n = (size_t)nx * ny * nz;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // node number
    if (q >= n) return;
    const int x = (int)(q % nx), y = (int)((q / nx) % ny), z = (int)(q / ((size_t)nx * ny));
    const size_t s = ((size_t)z * ny + y) * px + x;                    // its address
    auto at = [&](int xx, int yy, int zz) {
        return phi[((size_t)clampi(zz, nz) * ny + clampi(yy, ny)) * px + clampi(xx, nx)];
    };
    const T p0 = phi[s];
    const T pn[6] = {at(x + 1, y, z), at(x - 1, y, z), at(x, y + 1, z),
                     at(x, y - 1, z), at(x, y, z + 1), at(x, y, z - 1)};
    T a, Nx, Ny, Nz;
    aniso_terms(c, (pn[0] - pn[1]) * c.inv2dx, (pn[2] - pn[3]) * c.inv2dx, (pn[4] - pn[5]) * c.inv2dx,
                a, Nx, Ny, Nz);
    const T k = c.k, zA = T(0.5) * (T(1) + k), zB = T(0.5) * (T(1) - k);
    const T q0 = T(0.5) * (T(1) - p0);
    T wn[6], rn[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        wn[d] = frcp(zA - zB * pn[d]);
        rn[d] = T(0.5) * (T(1) - pn[d]) * wn[d];
    }
    const T u = U[s];
    const T Jx = c.D * ((rn[0] - rn[1]) * c.inv2dx + q0 * (wn[0] - wn[1]) * c.inv2dx) * u;
    const T Jy = c.D * ((rn[2] - rn[3]) * c.inv2dx + q0 * (wn[2] - wn[3]) * c.inv2dx) * u;
    const T Jz = c.D * ((rn[4] - rn[5]) * c.inv2dx + q0 * (wn[4] - wn[5]) * c.inv2dx) * u;
    const size_t nodes = (size_t)px * (size_t)ny * (size_t)nz;
    const T ax = c.advf ? c.advf[s] : c.adv[0], ay = c.advf ? c.advf[nodes + s] : c.adv[1],
            az = c.advf ? c.advf[2 * nodes + s] : c.adv[2];
    Unroll<0, L::Q>::run([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr T wi = T(L::w(I));
        const T eN = T(L::ex(I)) * Nx + T(L::ey(I)) * Ny + T(L::ez(I)) * Nz;
        const T eJ = T(L::ex(I)) * Jx + T(L::ey(I)) * Jy + T(L::ez(I)) * Jz;
        const size_t o = (size_t)I * c.np + s;
        if (parts & 1) g[o] = Codec<S>::enc(-wi * eN * c.cphi_e2);
        if (parts & 2) h[o * hs] = Codec<S>::enc((I == 0) ? T(0) : wi * eJ * c.jt);
        // f = w_i theta [1 + e_i . v dt / (e^2 dx)]: deviation w_i theta e_i . v'
        const T ev = T(L::ex(I)) * ax + T(L::ey(I)) * ay + T(L::ez(I)) * az;
        if (parts & 2) f[o * hs] = Codec<S>::enc(c.has_adv ? wi * th[s] * ev : T(0));
    });
}

// Full populations in FP64 (deviation + rest equilibrium) for inspection.
template <class L, class T, class S>
__global__ __launch_bounds__(256) void k_decode(const Coef<T> c, const S* __restrict__ pop, int es, int field,
                                                const T* __restrict__ phi, const T* __restrict__ U,
                                                const T* __restrict__ th, double* __restrict__ out) {
    const size_t n = (size_t)c.nx * c.ny * c.nz;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // node number (output index)
    if (q >= n) return;
    const size_t s = (q / c.nx) * c.px + q % c.nx;                      // its address
    const T zA = T(0.5) * (T(1) + c.k), zB = T(0.5) * (T(1) - c.k);
    Unroll<0, L::Q>::run([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr double wi = L::w(I);
        const double d = (double)(T)Codec<S>::dec(pop[((size_t)I * c.np + s) * es]);
        double ref;
        if (field == 0) {
            ref = wi * (double)phi[s];
        } else if (field == 1) {
            const double ru = (double)(r_of(phi[s], zA, zB) * U[s]);
            ref = (I == 0) ? (double)U[s] - (1.0 - wi) * ru : wi * ru;
        } else {
            ref = wi * (double)th[s];
        }
        out[(size_t)I * n + q] = d + ref;
    });
}

// ==========================================================================
// Streaming only (collision = identity) on raw bits: checks the pull index
// mapping and the wall rules.
// ==========================================================================
template <class L, class B>
__global__ __launch_bounds__(256) void k_stream_only(int nx, int ny, int nz, int px, int symm, long long np,
                                                     int es,   // element stride
                                                     const B* __restrict__ in, B* __restrict__ out) {
    const size_t n = (size_t)nx * ny * nz;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int x = (int)(q % nx), y = (int)((q / nx) % ny), z = (int)(q / ((size_t)nx * ny));
    const size_t s = ((size_t)z * ny + y) * px + x;
    Unroll<0, L::Q>::run([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const Src src = source<L, I>(x, y, z, nx, ny, nz, symm);
        const size_t si = ((size_t)src.sz * ny + src.sy) * px + src.sx;
        out[((size_t)I * np + s) * es] = in[((size_t)src.j * np + si) * es];
    });
}

// ==========================================================================
// FP64 reductions: per-block partials (wavefront shuffles, then LDS), then a
// single-block fixed-order final pass.  Deterministic for a given grid.
// ==========================================================================
enum { RV_SOLID = 0, RV_MASS, RV_ENTH, RV_SUMU, RV_SUMPHI, RV_BAD, RV_NSUM,   // sums
       RV_TIPX = RV_NSUM, RV_TIPY, RV_TIPZ, RV_PMAX, RV_NEG_PMIN, RV_COUNT };   // maxima
constexpr int RED_STRIDE = 16;   // doubles per partial / record slot
constexpr int RED_BLOCKS_NOALLOC = 1024;   // partial records of the allocation-free reduction

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

template <class T>
__global__ __launch_bounds__(256) void k_reduce_part(int nx, int ny, int nz, int px, double k, double dv,
                                                     const T* __restrict__ phi, const T* __restrict__ U,
                                                     const T* __restrict__ th, double* __restrict__ part) {
    __shared__ double sh[4][RV_COUNT];
    const size_t n = (size_t)nx * ny * nz;
    double v[RV_COUNT];
#pragma unroll
    for (int i = 0; i < RV_NSUM; ++i) v[i] = 0.0;
#pragma unroll
    for (int i = RV_NSUM; i < RV_COUNT; ++i) v[i] = -INFINITY;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(q % nx), y = (int)((q / nx) % ny), z = (int)(q / ((size_t)nx * ny));
        const size_t s = ((size_t)z * ny + y) * px + x;
        const double f = (double)phi[s], u = (double)U[s], t = (double)th[s];
        if (!isfinite(f) || !isfinite(u) || !isfinite(t)) {
            v[RV_BAD] += 1.0;
            continue;
        }
        v[RV_SOLID] += 0.5 * (1.0 + f);
        v[RV_MASS] += (0.5 * (1.0 + k) - 0.5 * (1.0 - k) * f) * (1.0 + (1.0 - k) * u) * dv;
        v[RV_ENTH] += (t - 0.5 * f) * dv;
        v[RV_SUMU] += u * dv;
        v[RV_SUMPHI] += f * dv;
        v[RV_PMAX] = fmax(v[RV_PMAX], f);
        v[RV_NEG_PMIN] = fmax(v[RV_NEG_PMIN], -f);
        if (f > 0.0) {
            if (x + 1 < nx) {
                const double fn = (double)phi[s + 1];
                if (fn <= 0.0) v[RV_TIPX] = fmax(v[RV_TIPX], x + f / (f - fn));
            }
            if (y + 1 < ny) {
                const double fn = (double)phi[s + px];
                if (fn <= 0.0) v[RV_TIPY] = fmax(v[RV_TIPY], y + f / (f - fn));
            }
            if (z + 1 < nz) {
                const double fn = (double)phi[s + (size_t)px * ny];
                if (fn <= 0.0) v[RV_TIPZ] = fmax(v[RV_TIPZ], z + f / (f - fn));
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < RV_COUNT; ++i) {
        const double r = i < RV_NSUM ? wave_sum(v[i]) : wave_max(v[i]);
        if (lane == 0) sh[wv][i] = r;
    }
    __syncthreads();
    if (threadIdx.x < RV_COUNT) {
        const int i = threadIdx.x;
        double r = sh[0][i];
        for (int w = 1; w < 4; ++w) r = i < RV_NSUM ? r + sh[w][i] : fmax(r, sh[w][i]);
        part[(size_t)blockIdx.x * RED_STRIDE + i] = r;
    }
}

// Element-wise type conversion of a field between row pitches (device-resident
// field I/O): rows of nx values, pin and pout elements apart.
template <class From, class To>
__global__ __launch_bounds__(256) void k_convert(const From* __restrict__ in, To* __restrict__ out, int nx,
                                                 int pin, int pout, size_t rows) {
    const size_t n = rows * (size_t)nx;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const size_t r = i / nx, x = i % nx;
        out[r * pout + x] = (To)in[r * pin + x];
    }
}

}  // namespace lbpf
