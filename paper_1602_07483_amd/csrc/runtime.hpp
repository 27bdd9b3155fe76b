// runtime.hpp -- host-side state and launch helpers shared by the library's
// translation units: lbpf.hip (the C ABI, initialisation, reductions,
// batches) and step.hip (the launches of the two step kernels, compiled once
// per lattice and storage type so that their instantiations build in
// parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbpf.h"
#include "kernels.hpp"

namespace lbpf_rt {

using namespace lbpf;

constexpr int HIST_CAP = 8192;
constexpr int RED_BLOCKS = 1024;
constexpr size_t kNoallocMaxNodes = (size_t)1 << 31;   // lbpf_reduce_fields_noalloc

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};

// Tile shapes (TX x TY threads, one node per thread; a wavefront covers
// 64/TX rows).
struct Shape {
    int tx, ty;
};
constexpr Shape kShapes[] = {{64, 2}, {64, 4}, {32, 4}, {32, 8}, {32, 16}};
constexpr int kNumShapes = 5;

// Is tile shape i available for a storage type?  FP64: 64 x 2 and 32 x 4.
inline bool shape_ok(int storage, int i) {
    if (storage == LBPF_F64) return i == 0 || i == 2;
    return i >= 0 && i < kNumShapes;
}

// The two step kernels, each with a launch of its own.
enum { K_PHI = 0, K_UT = 1 };

// Default launch per kernel and storage type (index: lbpf_storage), the
// fastest measured at 256^3 on D3Q19: k_phi on 32x8 tiles, k_ut on 64x4 tiles
// with FP32 populations (a 256-byte row keeps every line of an x-aligned pull
// within one block) and 32x8 with 16-bit ones; FP64 has 64x2 and 32x4 only.
// Tiles are dealt to the XCDs in contiguous runs except for FP32 k_ut, whose
// 64x4 tiles run 4 % faster in the hardware's round-robin order (although
// more of their reads then miss the XCD's L2).
constexpr int kDefaultShape[2][4] = {{3, 3, 3, 2}, {1, 3, 3, 2}};
constexpr int kDefaultZslab[2][4] = {{6, 6, 6, 4}, {6, 6, 6, 4}};
constexpr int kDefaultRemap[2][4] = {{1, 1, 1, 1}, {0, 1, 1, 1}};

// Padding added to the stride between population arrays: 17 x 256 bytes.
constexpr size_t kStridePadBytes = 17 * 256;
// The one k_ut tile with the advection-diffusion variant: 32x8 (FP64 32x4).
// Its wider halo terms (four values per node instead of one) would cost the
// 64x4 FP32 tile a block per CU.
constexpr int kAdvShape[4] = {3, 3, 3, 2};
const char* const kAdvTileMsg =
    "advection, skip_U and skip_theta run k_ut on its advection tile only (32x8; FP64 32x4)";

}  // namespace lbpf_rt

struct lbpf_ctx {
    lbpf_grid grid;
    lbpf_params prm;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool in_batch = false;   // member of a batch: stepped through lbpf_batch_step only
    int graph_steps = 0;     // >0: replay the step loop from a captured HIP graph
    hipGraphExec_t gexec = nullptr;
    int g_shape[2] = {-1, -1}, g_zslab[2] = {-1, -1}, g_remap[2] = {-1, -1}, g_cur = -1;
    int q = 19;              // lattice of g (phase field)
    int q_ut = 19;           // lattice of h and f (U, theta)
    int storage = LBPF_F32;
    size_t sbytes = 4;       // bytes per stored population
    size_t tbytes = 4;       // bytes per field value (compute type)
    size_t n = 0;            // nodes
    int px = 0;              // row pitch of the device arrays: nx rounded up to 32
    size_t na = 0;           // elements of one device field array, px * ny * nz
    size_t np = 0;           // population stride in elements (na rounded up to 64)
    void* pop[3][2] = {};    // [field][parity]
    // Element stride of h and f: 2 when both fields are solved and their
    // populations share one pair array (h at even, f at odd elements;
    // pop[2] is then pop[1] plus one element and owns no memory), else 1.
    int hs = 1;
    void* fld[3][2] = {};    // phi, U, theta [parity]
    int cur = 0;
    bool have_fields = false;
    int64_t step = 0;
    double* part = nullptr;  // RED_BLOCKS partials
    double* hist = nullptr;  // HIST_CAP records
    double* fresh = nullptr; // one record for lbpf_read
    void* vfield = nullptr;  // NULL, or the advective velocity field, [3][n] values of v dt/(e^2 dx)
    int64_t hist_count = 0;
    // launch of k_phi [0] and k_ut [1]: tile shape id (see kShapes), z slab,
    // XCD-chunked tile order
    int shape[2] = {3, 3};
    int zslab[2] = {4, 4};
    int remap[2] = {1, 1};
    bool timing = false;
    std::vector<lbpf_rt::TimedLaunch> launches;
    std::vector<hipEvent_t> pool;
    double t_ms[3] = {0, 0, 0};
    int64_t t_n[3] = {0, 0, 0};
    std::string err;
};

namespace lbpf_rt {

#define CHK(call)                                                                  \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);          \
            return LBPF_EDEVICE;                                                   \
        }                                                                          \
    } while (0)

// Records msg as the context's last error (the thread's creation error when
// ctx is NULL) and returns s.
lbpf_status fail(lbpf_ctx* ctx, lbpf_status s, const std::string& msg);

// Model constants of a context, with the tiling of kernel k.
template <class T>
Coef<T> make_coef(const lbpf_ctx* ctx, int k = K_PHI) {
    const lbpf_params& p = ctx->prm;
    const lbpf_grid& g = ctx->grid;
    // each scheme takes the e^2 of its own lattice
    const double e2g = lattice_e2(ctx->q), kE2 = lattice_e2(ctx->q_ut);
    const Shape sh = kShapes[ctx->shape[k]];
    Coef<T> c{};
    c.nx = g.nx; c.ny = g.ny; c.nz = g.nz;
    c.px = ctx->px;
    c.symm = 0;
    for (int f = 0; f < 6; ++f)
        if (g.wall[f] == LBPF_WALL_SYMMETRY) c.symm |= 1 << f;
    c.zslab = ctx->zslab[k];
    c.remap = ctx->remap[k];
    c.nbx = (g.nx + sh.tx - 1) / sh.tx;
    c.nby = (g.ny + sh.ty - 1) / sh.ty;
    c.nbz = (g.nz + ctx->zslab[k] - 1) / ctx->zslab[k];
    c.np = (long long)ctx->np;
    c.aniso = p.aniso;
    c.eps = (T)p.eps;
    c.delta = (T)p.delta;
    c.inv2dx = (T)(1.0 / (2.0 * p.dx));
    c.smin = (T)(1e-12 / (p.dx * p.dx));
    c.eta_c = (T)(p.W0 * p.W0 * p.dt / (e2g * p.tau0 * p.dx * p.dx));
    c.cphi_e2 = (T)(p.dt * p.W0 * p.W0 / (p.dx * p.tau0 * e2g));
    c.dt_tau0 = (T)(p.dt / p.tau0);
    c.lambda = (T)p.lambda;
    c.Mcinf = (T)p.Mcinf;
    c.k = (T)p.k;
    c.D = (T)p.D;
    c.inv_dt = (T)(1.0 / p.dt);
    c.inv_dx2 = (T)(1.0 / (p.dx * p.dx));
    c.jat_c = (T)(p.W0 / (2.0 * std::sqrt(2.0)));
    const double etaU = p.D * p.dt / (kE2 * p.dx * p.dx) + 0.5;
    const double etaT = p.kappa * p.dt / (kE2 * p.dx * p.dx) + 0.5;
    c.omU = (T)(1.0 / etaU);
    c.omT = (T)(1.0 / etaT);
    c.etaU = (T)etaU;
    c.dt = (T)p.dt;
    c.jcoef = (T)(p.dt / (kE2 * p.dx) / etaU);
    c.jt = (T)(p.dt / (kE2 * p.dx));
    c.has_adv = ctx->vfield != nullptr;
    c.advf = (const T*)ctx->vfield;
    for (int a = 0; a < 3; ++a) {
        c.adv[a] = (T)(p.vel[a] * p.dt / (kE2 * p.dx));
        if (p.vel[a] != 0.0) c.has_adv = 1;
    }
    return c;
}

inline bool has_advection(const lbpf_ctx* ctx) {
    return ctx->vfield != nullptr || ctx->prm.vel[0] != 0.0 || ctx->prm.vel[1] != 0.0 ||
           ctx->prm.vel[2] != 0.0;
}

// Lattice of field f's populations (0: phi; 1, 2: U, theta).
inline int lattice_of(const lbpf_ctx* ctx, int f) { return f == 0 ? ctx->q : ctx->q_ut; }

inline int default_shape(const lbpf_ctx* ctx, int k) { return kDefaultShape[k][ctx->storage]; }

// Element stride of field f's populations (1, or 2 for paired h and f).
inline int pop_stride(const lbpf_ctx* ctx, int f) { return f == 0 ? 1 : ctx->hs; }
// Bytes of the allocation that holds field f's populations, 0 where another
// field's allocation holds them (f of a pair).
inline size_t pop_alloc_bytes(const lbpf_ctx* ctx, int f) {
    if (f == 2 && ctx->hs == 2) return 0;
    return ctx->np * (size_t)lattice_of(ctx, f) * ctx->sbytes * (size_t)pop_stride(ctx, f);
}
// The allocation holding field f's populations at parity par, and the
// element offset of field f within each of its elements' strides.
inline void* pop_alloc(const lbpf_ctx* ctx, int f, int par) {
    return (f == 2 && ctx->hs == 2) ? ctx->pop[1][par] : ctx->pop[f][par];
}
inline int pop_lane(const lbpf_ctx* ctx, int f) { return (f == 2 && ctx->hs == 2) ? 1 : 0; }

inline int adv_shape(const lbpf_ctx* ctx) { return kAdvShape[ctx->storage]; }

// k_ut needs one of its variants (advection, theta alone or U alone), which
// exist on the advection tile only.
inline bool ut_pinned(const lbpf_ctx* ctx) {
    return has_advection(ctx) || ctx->prm.skip_U != 0 || ctx->prm.skip_theta != 0;
}

inline int total_tiles(const lbpf_ctx* ctx, int k) {
    const Shape sh = kShapes[ctx->shape[k]];
    const int nbx = (ctx->grid.nx + sh.tx - 1) / sh.tx;
    const int nby = (ctx->grid.ny + sh.ty - 1) / sh.ty;
    const int nbz = (ctx->grid.nz + ctx->zslab[k] - 1) / ctx->zslab[k];
    return nbx * nby * nbz;
}

inline hipEvent_t get_event(lbpf_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrapper: optional event pair around the launch.
template <class F>
lbpf_status timed(lbpf_ctx* ctx, int kind, F&& launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        a = get_event(ctx);
        b = get_event(ctx);
        if (!a || !b) return fail(ctx, LBPF_EDEVICE, "hipEventCreate failed");
        CHK(hipEventRecord(a, ctx->stream));
    }
    launch();
    CHK(hipGetLastError());
    if (ctx->timing) {
        CHK(hipEventRecord(b, ctx->stream));
        ctx->launches.push_back({kind, a, b});
    }
    return LBPF_OK;
}

// One time step (k_phi, then k_ut) of lattice L with compute type T and
// storage S; defined in step.hip, instantiated once per pair.
template <class L, class T, class S>
lbpf_status launch_step_s(lbpf_ctx* ctx);
// The two kernels alone, for a phase field and transport fields on different
// lattices (the caller flips the parity after both).
template <class L, class T, class S>
lbpf_status launch_phi_s(lbpf_ctx* ctx);
template <class L, class T, class S>
lbpf_status launch_ut_s(lbpf_ctx* ctx);
// One batch launch of k_phi (kernel K_PHI) or k_ut (K_UT) with tile shape id
// `shape` over nwork (domain, tile) work items, reading the populations and
// fields of parity par from the DomainDesc<T> array desc; defined in
// step.hip.  Returns a HIP error code.
template <class L, class T, class S>
hipError_t batch_launch_s(int kernel, int shape, const void* desc, const int2* work, int nwork, int par,
                          hipStream_t stream);

}  // namespace lbpf_rt
