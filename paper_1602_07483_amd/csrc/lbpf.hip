// lbpf.hip -- host runtime and C ABI (include/lbpf.h) of the gfx950
// lattice-Boltzmann phase-field library.
//
// Step order (Sec. 3.4, "Algorithm implementation"): the phase field first
// (kernel k_phi), then supersaturation and temperature with the new phase
// field (kernel k_ut).  Each field has two population lattices and two field
// buffers; the parity `cur` names the current state.
#include "runtime.hpp"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <mutex>

// Digest of the kernel sources this library was compiled from (set by the
// build); part of the key of persisted autotuner results.
#ifndef LBPF_KERNEL_BUILD
#define LBPF_KERNEL_BUILD "unknown"
#endif

// The library's two non-template kernels, defined in this translation unit
// only (the step translation units include kernels.hpp too).
namespace lbpf {

// A named range on the profiler's timeline (rocprofv3 --marker-trace) for
// the duration of one library call; free when no profiler is attached.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// Record layout (RED_STRIDE doubles): step, solid, mass, enthalpy, tip x,y,z,
// phi min, phi max, non-finite count, sum U, sum phi.
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int nparts,
                                                      double inv_n, double cx, double cy, double cz,
                                                      long long step, double* __restrict__ rec) {
    __shared__ double sh[4][RV_COUNT];
    double v[RV_COUNT];
#pragma unroll
    for (int i = 0; i < RV_NSUM; ++i) v[i] = 0.0;
#pragma unroll
    for (int i = RV_NSUM; i < RV_COUNT; ++i) v[i] = -INFINITY;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
#pragma unroll
        for (int i = 0; i < RV_COUNT; ++i) {
            const double x = part[(size_t)p * RED_STRIDE + i];
            v[i] = i < RV_NSUM ? v[i] + x : fmax(v[i], x);
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < RV_COUNT; ++i) {
        const double r = i < RV_NSUM ? wave_sum(v[i]) : wave_max(v[i]);
        if (lane == 0) sh[wv][i] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[RV_COUNT];
        for (int i = 0; i < RV_COUNT; ++i) {
            r[i] = sh[0][i];
            for (int w = 1; w < 4; ++w) r[i] = i < RV_NSUM ? r[i] + sh[w][i] : fmax(r[i], sh[w][i]);
        }
        const double nanv = __longlong_as_double(0x7ff8000000000000LL);
        rec[0] = (double)step;
        rec[1] = r[RV_SOLID] * inv_n;
        rec[2] = r[RV_MASS];
        rec[3] = r[RV_ENTH];
        rec[4] = r[RV_TIPX] > -1e300 ? r[RV_TIPX] - cx : nanv;
        rec[5] = r[RV_TIPY] > -1e300 ? r[RV_TIPY] - cy : nanv;
        rec[6] = r[RV_TIPZ] > -1e300 ? r[RV_TIPZ] - cz : nanv;
        rec[7] = -r[RV_NEG_PMIN];
        rec[8] = r[RV_PMAX];
        rec[9] = r[RV_BAD];
        rec[10] = r[RV_SUMU];
        rec[11] = r[RV_SUMPHI];
    }
}

// Bandwidth reference kernels: read-only (MODE 0), write-only (1) and copy
// (2) over n elements of V (2, 4, 8 or 16 bytes per lane), four accesses in
// flight per thread, optionally with streaming (non-temporal) hints, on a
// grid-stride loop.  The read-only form folds what it reads into one word per
// thread and stores it only when it equals a run-time value (all ones, which
// no fold of the zero-filled buffers reaches), so the loads cannot be removed.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned fold(unsigned short v) { return v; }
__device__ __forceinline__ unsigned fold(unsigned v) { return v; }
__device__ __forceinline__ unsigned fold(u32x2 v) { return v.x ^ v.y; }
__device__ __forceinline__ unsigned fold(u32x4 v) { return v.x ^ v.y ^ v.z ^ v.w; }
template <class V> __device__ __forceinline__ V splat(unsigned v) { return V(v); }
template <> __device__ __forceinline__ unsigned short splat<unsigned short>(unsigned v) { return (unsigned short)v; }

template <class V, int MODE, bool NT>
__global__ __launch_bounds__(256) void k_bw(const V* __restrict__ src, V* __restrict__ dst, size_t n,
                                            unsigned* __restrict__ sink, unsigned magic) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned acc = 0;
    auto ld = [&](size_t j) -> V {
        if constexpr (NT) return __builtin_nontemporal_load(&src[j]);
        else return src[j];
    };
    auto st = [&](size_t j, V v) {
        if constexpr (NT) __builtin_nontemporal_store(v, &dst[j]);
        else dst[j] = v;
    };
    for (; i + 3 * stride < n; i += 4 * stride) {
        V v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = MODE == 1 ? splat<V>((unsigned)(i + u * stride)) : ld(i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if constexpr (MODE == 0) acc ^= fold(v[u]);
            else st(i + u * stride, v[u]);
        }
    }
    for (; i < n; i += stride) {
        if constexpr (MODE == 0) acc ^= fold(ld(i));
        else st(i, MODE == 1 ? splat<V>((unsigned)i) : ld(i));
    }
    if (MODE == 0 && acc == magic) sink[0] = acc;
}

template <class V, int MODE>
void launch_bw(int nt, int nb, hipStream_t st, const void* src, void* dst, size_t n) {
    if (nt)
        hipLaunchKernelGGL((k_bw<V, MODE, true>), dim3(nb), dim3(256), 0, st, (const V*)src, (V*)dst, n,
                           (unsigned*)dst, 0xFFFFFFFFu);
    else
        hipLaunchKernelGGL((k_bw<V, MODE, false>), dim3(nb), dim3(256), 0, st, (const V*)src, (V*)dst, n,
                           (unsigned*)dst, 0xFFFFFFFFu);
}
template <class V>
void launch_bw_mode(int mode, int nt, int nb, hipStream_t st, const void* src, void* dst, size_t n) {
    if (mode == 0) launch_bw<V, 0>(nt, nb, st, src, dst, n);
    else if (mode == 1) launch_bw<V, 1>(nt, nb, st, src, dst, n);
    else launch_bw<V, 2>(nt, nb, st, src, dst, n);
}

}  // namespace lbpf

// Scratch of the reduction entry point that allocates nothing
// (lbpf_reduce_fields_noalloc): the per-block partial records of
// k_reduce_part, RED_BLOCKS x RED_STRIDE doubles (128 KiB) on every device
// the library runs on, held until the process ends.  Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device (scratch_on_device).
static __device__ __align__(256) double scratch[lbpf::RED_BLOCKS_NOALLOC * lbpf::RED_STRIDE];

using namespace lbpf;
using namespace lbpf_rt;

namespace {
// Device address of `scratch` on each device, taken once per device with that
// device current (each device holds its own copy of the array).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

namespace {
thread_local std::string g_create_error;
}  // namespace

lbpf_status lbpf_rt::fail(lbpf_ctx* ctx, lbpf_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return s;
}

// --------------------------------------------------------------------------
// Batch: independent domains stepped together by one launch per lattice type
// and kernel (optionally replayed from a captured graph).
// --------------------------------------------------------------------------
struct lbpf_batch {
    std::vector<lbpf_ctx*> dom;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int storage = LBPF_F32;
    int shape[2] = {3, 3}, zslab[2] = {6, 6};   // tile shape id and z slab of k_phi [0], k_ut [1]
    void* d_desc = nullptr;        // DomainDesc<T>[ndom]
    // work tables of k_phi [0] and k_ut [1] over the domains whose phi
    // (resp. U, theta) lattice is D3Q7, D3Q15, D3Q19
    int2* d_work[2][3] = {};
    int nwork[2][3] = {};
    bool built = false;
    int graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    int g_cur = -1;
    std::string err;
};

namespace {


// part 0: the whole step on one lattice; 1: k_phi alone; 2: k_ut alone
template <class L>
lbpf_status launch_step_l(lbpf_ctx* ctx, int part) {
    switch (ctx->storage) {
        case LBPF_F32:
            return part == 0 ? launch_step_s<L, float, float>(ctx)
                             : part == 1 ? launch_phi_s<L, float, float>(ctx) : launch_ut_s<L, float, float>(ctx);
        case LBPF_F16_DEV:
            return part == 0 ? launch_step_s<L, float, __half>(ctx)
                             : part == 1 ? launch_phi_s<L, float, __half>(ctx) : launch_ut_s<L, float, __half>(ctx);
        case LBPF_BF16_DEV:
            return part == 0   ? launch_step_s<L, float, __hip_bfloat16>(ctx)
                   : part == 1 ? launch_phi_s<L, float, __hip_bfloat16>(ctx)
                               : launch_ut_s<L, float, __hip_bfloat16>(ctx);
        case LBPF_F64:
            return part == 0 ? launch_step_s<L, double, double>(ctx)
                             : part == 1 ? launch_phi_s<L, double, double>(ctx) : launch_ut_s<L, double, double>(ctx);
    }
    return fail(ctx, LBPF_EINVAL, "bad storage");
}

lbpf_status launch_step_q(lbpf_ctx* ctx, int q, int part) {
    switch (q) {
        case 7: return launch_step_l<D3Q7>(ctx, part);
        case 15: return launch_step_l<D3Q15>(ctx, part);
        default: return launch_step_l<D3Q19>(ctx, part);
    }
}

lbpf_status launch_step(lbpf_ctx* ctx) {
    if (ctx->q_ut == ctx->q) return launch_step_q(ctx, ctx->q, 0);
    // phase field and transport fields on different lattices (Sec. 4.1's 2D validation)
    lbpf_status st = launch_step_q(ctx, ctx->q, 1);
    if (!st) st = launch_step_q(ctx, ctx->q_ut, 2);
    if (!st) ctx->cur = 1 - ctx->cur;
    return st;
}

// Initial populations of the sets whose lattice is L.
template <class L, class T, class S>
lbpf_status launch_init_t(lbpf_ctx* ctx) {
    const Coef<T> c = make_coef<T>(ctx);
    const int nb = (int)((ctx->n + 255) / 256);
    const int a = ctx->cur;
    const int parts = (ctx->q == L::Q ? 1 : 0) | (ctx->q_ut == L::Q ? 2 : 0);
    hipLaunchKernelGGL((k_init<L, T, S>), dim3(nb), dim3(256), 0, ctx->stream, c, (S*)ctx->pop[0][a],
                       (S*)ctx->pop[1][a], (S*)ctx->pop[2][a], ctx->hs, (const T*)ctx->fld[0][a],
                       (const T*)ctx->fld[1][a], (const T*)ctx->fld[2][a], parts);
    CHK(hipGetLastError());
    return LBPF_OK;
}

template <class L, class T, class S>
lbpf_status launch_decode_t(lbpf_ctx* ctx, int field, double* dout) {
    const Coef<T> c = make_coef<T>(ctx);
    const int nb = (int)((ctx->n + 255) / 256);
    const int a = ctx->cur;
    hipLaunchKernelGGL((k_decode<L, T, S>), dim3(nb), dim3(256), 0, ctx->stream, c,
                       (const S*)ctx->pop[field][a], pop_stride(ctx, field), field, (const T*)ctx->fld[0][a],
                       (const T*)ctx->fld[1][a], (const T*)ctx->fld[2][a], dout);
    CHK(hipGetLastError());
    return LBPF_OK;
}

template <class L, class T, class S>
lbpf_status by_storage_init(lbpf_ctx* ctx, int what, int field, double* dout) {
    return what == 0 ? launch_init_t<L, T, S>(ctx) : launch_decode_t<L, T, S>(ctx, field, dout);
}

template <class L>
lbpf_status init_or_decode_l(lbpf_ctx* ctx, int what, int field, double* dout) {
    switch (ctx->storage) {
        case LBPF_F32: return by_storage_init<L, float, float>(ctx, what, field, dout);
        case LBPF_F16_DEV: return by_storage_init<L, float, __half>(ctx, what, field, dout);
        case LBPF_BF16_DEV: return by_storage_init<L, float, __hip_bfloat16>(ctx, what, field, dout);
        case LBPF_F64: return by_storage_init<L, double, double>(ctx, what, field, dout);
    }
    return fail(ctx, LBPF_EINVAL, "bad storage");
}

lbpf_status init_or_decode_q(lbpf_ctx* ctx, int q, int what, int field, double* dout) {
    switch (q) {
        case 7: return init_or_decode_l<D3Q7>(ctx, what, field, dout);
        case 15: return init_or_decode_l<D3Q15>(ctx, what, field, dout);
        default: return init_or_decode_l<D3Q19>(ctx, what, field, dout);
    }
}

// what 0: initial populations of every set (one launch per lattice in use);
// what 1: decode one field's populations on its lattice.
lbpf_status init_or_decode(lbpf_ctx* ctx, int what, int field, double* dout) {
    if (what == 1) return init_or_decode_q(ctx, field == 0 ? ctx->q : ctx->q_ut, 1, field, dout);
    lbpf_status st = init_or_decode_q(ctx, ctx->q, 0, field, dout);
    if (!st && ctx->q_ut != ctx->q) st = init_or_decode_q(ctx, ctx->q_ut, 0, field, dout);
    return st;
}

// Streams the population sets of the fields in [f0, f1) on lattice L.
template <class L, class B>
lbpf_status stream_only_t(lbpf_ctx* ctx, int f0, int f1) {
    int symm = 0;
    for (int f = 0; f < 6; ++f)
        if (ctx->grid.wall[f] == LBPF_WALL_SYMMETRY) symm |= 1 << f;
    const int nb = (int)((ctx->n + 255) / 256);
    const int a = ctx->cur, b = 1 - ctx->cur;
    for (int f = f0; f < f1; ++f)
        hipLaunchKernelGGL((k_stream_only<L, B>), dim3(nb), dim3(256), 0, ctx->stream, ctx->grid.nx,
                           ctx->grid.ny, ctx->grid.nz, ctx->px, symm, (long long)ctx->np,
                           pop_stride(ctx, f), (const B*)ctx->pop[f][a], (B*)ctx->pop[f][b]);
    CHK(hipGetLastError());
    return LBPF_OK;
}

// The fields follow the populations' parity unchanged.
lbpf_status stream_only_fields(lbpf_ctx* ctx) {
    const int a = ctx->cur, b = 1 - ctx->cur;
    // the fields follow the populations' parity unchanged
    for (int f = 0; f < 3; ++f)
        CHK(hipMemcpyAsync(ctx->fld[f][b], ctx->fld[f][a], ctx->na * ctx->tbytes,
                           hipMemcpyDeviceToDevice, ctx->stream));
    ctx->cur = b;
    return LBPF_OK;
}

template <class L>
lbpf_status stream_only_l(lbpf_ctx* ctx, int f0, int f1) {
    switch (ctx->sbytes) {
        case 2: return stream_only_t<L, uint16_t>(ctx, f0, f1);
        case 4: return stream_only_t<L, uint32_t>(ctx, f0, f1);
        case 8: return stream_only_t<L, uint64_t>(ctx, f0, f1);
    }
    return fail(ctx, LBPF_EINVAL, "bad storage");
}

lbpf_status stream_only_q(lbpf_ctx* ctx, int q, int f0, int f1) {
    switch (q) {
        case 7: return stream_only_l<D3Q7>(ctx, f0, f1);
        case 15: return stream_only_l<D3Q15>(ctx, f0, f1);
        default: return stream_only_l<D3Q19>(ctx, f0, f1);
    }
}

template <class T>
lbpf_status launch_reduce_t(lbpf_ctx* ctx, double* rec) {
    const lbpf_params& p = ctx->prm;
    const int a = ctx->cur;
    const int nb = (int)std::min<size_t>(RED_BLOCKS, (ctx->n + 255) / 256);
    lbpf_status st = timed(ctx, 2, [&] {
        hipLaunchKernelGGL((k_reduce_part<T>), dim3(nb), dim3(256), 0, ctx->stream, ctx->grid.nx,
                           ctx->grid.ny, ctx->grid.nz, ctx->px, p.k, p.dx * p.dx * p.dx,
                           (const T*)ctx->fld[0][a], (const T*)ctx->fld[1][a],
                           (const T*)ctx->fld[2][a], ctx->part);
    });
    if (st) return st;
    return timed(ctx, 2, [&] {
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, ctx->stream, ctx->part, nb,
                           1.0 / (double)ctx->n, p.centre[0], p.centre[1], p.centre[2],
                           (long long)ctx->step, rec);
    });
}

lbpf_status launch_reduce(lbpf_ctx* ctx, double* rec) {
    return ctx->storage == LBPF_F64 ? launch_reduce_t<double>(ctx, rec)
                                    : launch_reduce_t<float>(ctx, rec);
}

void unpack_record(const double* r, lbpf_reductions* out) {
    out->step = (int64_t)r[0];
    out->solid_fraction = r[1];
    out->solute_mass = r[2];
    out->enthalpy = r[3];
    out->tip[0] = r[4]; out->tip[1] = r[5]; out->tip[2] = r[6];
    out->phi_min = r[7];
    out->phi_max = r[8];
    out->nonfinite = r[9];
    out->sum_U = r[10];
    out->sum_phi = r[11];
    for (int a = 0; a < 3; ++a) out->tip_vel[a] = std::nan("");
}

// Tip velocity of cur from the record prev made before it (physical units).
void set_tip_vel(lbpf_reductions* cur, const lbpf_reductions& prev, const lbpf_params& p) {
    if (cur->step <= prev.step) return;
    const double s = p.dx / ((double)(cur->step - prev.step) * p.dt);
    for (int a = 0; a < 3; ++a) cur->tip_vel[a] = (cur->tip[a] - prev.tip[a]) * s;
}

bool healthy(const lbpf_reductions& r) {
    return r.nonfinite == 0.0 && r.phi_max <= 1.0 + 1e-3 && r.phi_min >= -1.0 - 1e-3;
}

// Host staging between the caller's packed rows (nx values) and the device
// layout (rows px values apart): one linear copy instead of a copy per row.
void pack_rows(void* dst, const void* src, size_t row_bytes, size_t pitch_bytes, size_t rows) {
    for (size_t r = 0; r < rows; ++r)
        std::memcpy((char*)dst + r * pitch_bytes, (const char*)src + r * row_bytes, row_bytes);
}
void unpack_rows(void* dst, const void* src, size_t row_bytes, size_t pitch_bytes, size_t rows) {
    for (size_t r = 0; r < rows; ++r)
        std::memcpy((char*)dst + r * row_bytes, (const char*)src + r * pitch_bytes, row_bytes);
}

// Waits for the stream and moves the recorded launch events back to the
// pool, adding their durations to ms[kind] and counts to n[kind] when given.
lbpf_status drain_launches(lbpf_ctx* ctx, double* ms, int64_t* n) {
    CHK(hipStreamSynchronize(ctx->stream));
    lbpf_status st = LBPF_OK;
    for (auto& l : ctx->launches) {
        if (ms && !st) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, l.a, l.b) != hipSuccess) st = fail(ctx, LBPF_EDEVICE, "event timing");
            ms[l.kind] += t;
            n[l.kind] += 1;
        }
        ctx->pool.push_back(l.a);
        ctx->pool.push_back(l.b);
    }
    ctx->launches.clear();
    return st;
}

void free_all(lbpf_ctx* ctx) {
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    for (int f = 0; f < 3; ++f)
        for (int p = 0; p < 2; ++p) {
            if (ctx->pop[f][p] && pop_alloc_bytes(ctx, f)) (void)hipFree(ctx->pop[f][p]);
            if (ctx->fld[f][p]) (void)hipFree(ctx->fld[f][p]);
        }
    for (int f = 0; f < 3; ++f)
        for (int p = 0; p < 2; ++p) ctx->pop[f][p] = ctx->fld[f][p] = nullptr;
    if (ctx->part) (void)hipFree(ctx->part);
    if (ctx->hist) (void)hipFree(ctx->hist);
    if (ctx->fresh) (void)hipFree(ctx->fresh);
    if (ctx->vfield) (void)hipFree(ctx->vfield);
    ctx->part = ctx->hist = ctx->fresh = nullptr;
    ctx->vfield = nullptr;
    for (auto& l : ctx->launches) {
        (void)hipEventDestroy(l.a);
        (void)hipEventDestroy(l.b);
    }
    ctx->launches.clear();
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    ctx->pool.clear();
}

}  // namespace

extern "C" {

int32_t lbpf_storage_bytes(int32_t storage) {
    switch (storage) {
        case LBPF_F32: return 4;
        case LBPF_F16_DEV: return 2;
        case LBPF_BF16_DEV: return 2;
        case LBPF_F64: return 8;
    }
    return 0;
}

const char* lbpf_last_error(const lbpf_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

lbpf_status lbpf_create(const lbpf_grid* grid, const lbpf_params* params, void* hip_stream,
                        lbpf_ctx** out) {
    if (!out) return fail(nullptr, LBPF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grid || !params) return fail(nullptr, LBPF_EINVAL, "grid or params is NULL");
    const lbpf_grid& g = *grid;
    const lbpf_params& p = *params;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return fail(nullptr, LBPF_EINVAL, "grid size < 1");
    if ((double)g.nx * g.ny * g.nz > 2.0e9) return fail(nullptr, LBPF_EINVAL, "grid too large");
    if (g.lattice != LBPF_D3Q7 && g.lattice != LBPF_D3Q15 && g.lattice != LBPF_D3Q19)
        return fail(nullptr, LBPF_EINVAL, "lattice must be 7, 15 or 19");
    if (g.lattice_ut != 0 && g.lattice_ut != LBPF_D3Q7 && g.lattice_ut != LBPF_D3Q15 &&
        g.lattice_ut != LBPF_D3Q19)
        return fail(nullptr, LBPF_EINVAL, "lattice_ut must be 0, 7, 15 or 19");
    if (lbpf_storage_bytes(g.storage) == 0) return fail(nullptr, LBPF_EINVAL, "bad storage");
    for (int f = 0; f < 6; ++f)
        if (g.wall[f] != LBPF_WALL_NOFLUX && g.wall[f] != LBPF_WALL_SYMMETRY)
            return fail(nullptr, LBPF_EINVAL, "bad wall type");
    if (!(p.dx > 0) || !(p.dt > 0) || !(p.W0 > 0) || !(p.tau0 > 0))
        return fail(nullptr, LBPF_EINVAL, "dx, dt, W0 and tau0 must be > 0");
    if (!(p.k > 0 && p.k < 1)) return fail(nullptr, LBPF_EINVAL, "k must lie in (0,1)");
    if (!(p.D >= 0) || !(p.kappa >= 0)) return fail(nullptr, LBPF_EINVAL, "D, kappa must be >= 0");
    if (!(p.eps >= 0 && p.eps <= 0.25) || !std::isfinite(p.delta) || !std::isfinite(p.lambda) ||
        !std::isfinite(p.Mcinf))
        return fail(nullptr, LBPF_EINVAL, "bad anisotropy or coupling parameter");
    if (p.aniso != LBPF_ANISO_CUBIC && p.aniso != LBPF_ANISO_K41K61)
        return fail(nullptr, LBPF_EINVAL, "bad anisotropy function");
    if (p.reduce_every < 0) return fail(nullptr, LBPF_EINVAL, "reduce_every < 0");
    if (!std::isfinite(p.vel[0]) || !std::isfinite(p.vel[1]) || !std::isfinite(p.vel[2]))
        return fail(nullptr, LBPF_EINVAL, "advective velocity must be finite");
    if (p.skip_U != 0 && p.skip_U != 1) return fail(nullptr, LBPF_EINVAL, "skip_U must be 0 or 1");
    if (p.skip_U && p.Mcinf != 0.0)
        return fail(nullptr, LBPF_EINVAL, "skip_U needs Mcinf = 0 (otherwise U acts on phi)");
    if (p.skip_theta != 0 && p.skip_theta != 1) return fail(nullptr, LBPF_EINVAL, "skip_theta must be 0 or 1");
    if (p.skip_theta && p.skip_U) return fail(nullptr, LBPF_EINVAL, "skip_U and skip_theta leave nothing to solve");
    if (p.skip_theta && (p.vel[0] != 0.0 || p.vel[1] != 0.0 || p.vel[2] != 0.0))
        return fail(nullptr, LBPF_EINVAL, "advection needs the heat equation (skip_theta = 0)");

    lbpf_ctx* ctx = new (std::nothrow) lbpf_ctx();
    if (!ctx) return fail(nullptr, LBPF_ENOMEM, "host allocation failed");
    ctx->grid = g;
    ctx->prm = p;
    ctx->stream = (hipStream_t)hip_stream;
    if (!ctx->stream) {
        // capture needs a stream other than the null stream: own one
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return fail(nullptr, LBPF_EDEVICE, "hipStreamCreateWithFlags failed");
        }
        ctx->own_stream = true;
    }
    ctx->q = g.lattice;
    ctx->q_ut = g.lattice_ut ? g.lattice_ut : g.lattice;
    ctx->storage = g.storage;
    ctx->sbytes = (size_t)lbpf_storage_bytes(g.storage);
    ctx->tbytes = g.storage == LBPF_F64 ? 8 : 4;
    for (int k = 0; k < 2; ++k) {
        ctx->shape[k] = kDefaultShape[k][g.storage];
        ctx->zslab[k] = kDefaultZslab[k][g.storage];
        ctx->remap[k] = kDefaultRemap[k][g.storage];
    }
    if (ut_pinned(ctx)) ctx->shape[K_UT] = adv_shape(ctx);
    ctx->n = (size_t)g.nx * g.ny * g.nz;
    // rows start on 128-byte lines (FP32): a tile row then reads whole lines
    ctx->px = (g.nx + 31) / 32 * 32;
    ctx->na = (size_t)ctx->px * g.ny * g.nz;
    // Stride between the Q arrays of a field: whole 64-element groups, plus
    // an odd number of 256-byte units, so that the Q loads of one node do not
    // sit a power of two apart (at 256^3 that power of two is 64 MiB, and
    // k_phi FP32 runs 3.5 % slower on it).
    ctx->np = (ctx->na + 63) / 64 * 64 + kStridePadBytes / ctx->sbytes;
    // h and f of a node and direction are pulled from the same source: with
    // both fields solved they share one pair array, loaded and stored by k_ut
    // with one instruction per direction
    ctx->hs = (p.skip_U == 0 && p.skip_theta == 0) ? 2 : 1;
    hipError_t e = hipSuccess;
    for (int f = 0; f < 3 && e == hipSuccess; ++f)
        for (int par = 0; par < 2 && e == hipSuccess; ++par) {
            if (pop_alloc_bytes(ctx, f))
                e = hipMalloc(&ctx->pop[f][par], pop_alloc_bytes(ctx, f));
            else
                ctx->pop[f][par] = (char*)ctx->pop[1][par] + ctx->sbytes;   // f: the odd elements
            if (e == hipSuccess) e = hipMalloc(&ctx->fld[f][par], ctx->na * ctx->tbytes);
        }
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->part, RED_BLOCKS * RED_STRIDE * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->hist, (size_t)HIST_CAP * RED_STRIDE * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->fresh, RED_STRIDE * sizeof(double));
    if (e != hipSuccess) {
        const lbpf_status s = e == hipErrorOutOfMemory ? LBPF_ENOMEM : LBPF_EDEVICE;
        const std::string msg = std::string("device allocation: ") + hipGetErrorString(e);
        free_all(ctx);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return fail(nullptr, s, msg);
    }
    *out = ctx;
    return LBPF_OK;
}

lbpf_status lbpf_destroy(lbpf_ctx* ctx) {
    if (!ctx) return LBPF_OK;
    if (ctx->in_batch) return fail(ctx, LBPF_ESTATE, "context belongs to a batch");
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return LBPF_OK;
}

lbpf_status lbpf_set_fields(lbpf_ctx* ctx, const double* phi, const double* U, const double* theta) {
    const lbpf::Range range("lbpf_set_fields");
    if (!ctx) return LBPF_EINVAL;
    if (!phi || !U || !theta) return fail(ctx, LBPF_EINVAL, "NULL field array");
    ctx->cur = 0;
    const double* src[3] = {phi, U, theta};
    for (int f = 0; f < 3; ++f) {
        const size_t nx = ctx->grid.nx, px = ctx->px, rows = (size_t)ctx->grid.ny * ctx->grid.nz;
        if (ctx->tbytes == 8) {
            std::vector<double> tmp(ctx->na, 0.0);
            pack_rows(tmp.data(), src[f], nx * 8, px * 8, rows);
            CHK(hipMemcpyAsync(ctx->fld[f][0], tmp.data(), ctx->na * 8, hipMemcpyHostToDevice, ctx->stream));
            CHK(hipStreamSynchronize(ctx->stream));
        } else {
            std::vector<float> tmp(ctx->na, 0.f);
            for (size_t r = 0; r < rows; ++r)
                for (size_t x = 0; x < nx; ++x) tmp[r * px + x] = (float)src[f][r * nx + x];
            CHK(hipMemcpyAsync(ctx->fld[f][0], tmp.data(), ctx->na * 4, hipMemcpyHostToDevice, ctx->stream));
            CHK(hipStreamSynchronize(ctx->stream));
        }
    }
    lbpf_status st = init_or_decode(ctx, 0, 0, nullptr);
    if (st) return st;
    CHK(hipStreamSynchronize(ctx->stream));
    ctx->have_fields = true;
    ctx->step = 0;
    ctx->hist_count = 0;
    return LBPF_OK;
}

// Capture graph_steps (even) steps starting from the current parity; the
// parity is the same again after the graph, so the graph is replayable.
lbpf_status capture_graph(lbpf_ctx* ctx) {
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    const int cur0 = ctx->cur;
    const bool was = ctx->timing;
    ctx->timing = false;
    hipGraph_t g = nullptr;
    CHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    lbpf_status st = LBPF_OK;
    for (int k = 0; k < ctx->graph_steps && !st; ++k) st = launch_step(ctx);
    const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    ctx->timing = was;
    ctx->cur = cur0;
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(ctx, LBPF_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        ctx->gexec = nullptr;
        return fail(ctx, LBPF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    for (int k = 0; k < 2; ++k) {
        ctx->g_shape[k] = ctx->shape[k];
        ctx->g_zslab[k] = ctx->zslab[k];
        ctx->g_remap[k] = ctx->remap[k];
    }
    ctx->g_cur = cur0;
    return LBPF_OK;
}

lbpf_status lbpf_step(lbpf_ctx* ctx, int64_t nsteps) {
    const lbpf::Range range("lbpf_step");
    if (!ctx) return LBPF_EINVAL;
    if (nsteps < 0) return fail(ctx, LBPF_EINVAL, "nsteps < 0");
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    if (ctx->in_batch) return fail(ctx, LBPF_ESTATE, "context belongs to a batch; use lbpf_batch_step");
    const int R = ctx->prm.reduce_every;
    const int G = ctx->graph_steps;
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t to_red = R > 0 ? R - ctx->step % R : left;
        if (G > 0 && !ctx->timing && std::min(left, to_red) >= G) {
            bool same = ctx->gexec && ctx->g_cur == ctx->cur;
            for (int k = 0; k < 2; ++k)
                same = same && ctx->g_shape[k] == ctx->shape[k] && ctx->g_zslab[k] == ctx->zslab[k] &&
                       ctx->g_remap[k] == ctx->remap[k];
            if (!same) {
                lbpf_status st = capture_graph(ctx);
                if (st) return st;
            }
            CHK(hipGraphLaunch(ctx->gexec, ctx->stream));
            ctx->step += G;
            left -= G;
        } else {
            lbpf_status st = launch_step(ctx);
            if (st) return st;
            ctx->step++;
            left--;
        }
        if (R > 0 && ctx->step % R == 0) {
            double* rec = ctx->hist + (size_t)(ctx->hist_count % HIST_CAP) * RED_STRIDE;
            lbpf_status st = launch_reduce(ctx, rec);
            if (st) return st;
            ctx->hist_count++;
        }
    }
    return LBPF_OK;
}

lbpf_status lbpf_set_graph(lbpf_ctx* ctx, int32_t steps_per_graph) {
    if (!ctx) return LBPF_EINVAL;
    if (steps_per_graph < 0 || (steps_per_graph % 2) != 0)
        return fail(ctx, LBPF_EINVAL, "steps_per_graph must be 0 or a positive even number");
    ctx->graph_steps = steps_per_graph;
    if (ctx->gexec) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    return LBPF_OK;
}

lbpf_status lbpf_sync(lbpf_ctx* ctx) {
    if (!ctx) return LBPF_EINVAL;
    CHK(hipStreamSynchronize(ctx->stream));
    if (ctx->hist_count > 0) {
        double r[RED_STRIDE];
        const double* rec = ctx->hist + (size_t)((ctx->hist_count - 1) % HIST_CAP) * RED_STRIDE;
        CHK(hipMemcpy(r, rec, sizeof(r), hipMemcpyDeviceToHost));
        lbpf_reductions red;
        unpack_record(r, &red);
        if (!healthy(red))
            return fail(ctx, LBPF_EUNSTABLE, "health check failed at step " + std::to_string(red.step));
    }
    return LBPF_OK;
}

lbpf_status lbpf_read(lbpf_ctx* ctx, double* phi, double* U, double* theta, lbpf_reductions* red) {
    const lbpf::Range range("lbpf_read");
    if (!ctx) return LBPF_EINVAL;
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    double* dst[3] = {phi, U, theta};
    CHK(hipStreamSynchronize(ctx->stream));
    for (int f = 0; f < 3; ++f) {
        if (!dst[f]) continue;
        const size_t nx = ctx->grid.nx, px = ctx->px, rows = (size_t)ctx->grid.ny * ctx->grid.nz;
        if (ctx->tbytes == 8) {
            std::vector<double> tmp(ctx->na);
            CHK(hipMemcpy(tmp.data(), ctx->fld[f][ctx->cur], ctx->na * 8, hipMemcpyDeviceToHost));
            unpack_rows(dst[f], tmp.data(), nx * 8, px * 8, rows);
        } else {
            std::vector<float> tmp(ctx->na);
            CHK(hipMemcpy(tmp.data(), ctx->fld[f][ctx->cur], ctx->na * 4, hipMemcpyDeviceToHost));
            for (size_t r = 0; r < rows; ++r)
                for (size_t x = 0; x < nx; ++x) dst[f][r * nx + x] = (double)tmp[r * px + x];
        }
    }
    if (red) {
        const bool was = ctx->timing;
        ctx->timing = false;
        lbpf_status st = launch_reduce(ctx, ctx->fresh);
        ctx->timing = was;
        if (st) return st;
        double r[RED_STRIDE];
        CHK(hipMemcpyAsync(r, ctx->fresh, sizeof(r), hipMemcpyDeviceToHost, ctx->stream));
        CHK(hipStreamSynchronize(ctx->stream));
        unpack_record(r, red);
        // tip velocity against the latest history record made before this step
        for (int64_t back = 1; back <= 2 && back <= ctx->hist_count && back <= HIST_CAP; ++back) {
            double h[RED_STRIDE];
            CHK(hipMemcpy(h, ctx->hist + (size_t)((ctx->hist_count - back) % HIST_CAP) * RED_STRIDE, sizeof(h),
                          hipMemcpyDeviceToHost));
            lbpf_reductions prev;
            unpack_record(h, &prev);
            if (prev.step < red->step) {
                set_tip_vel(red, prev, ctx->prm);
                break;
            }
        }
        if (!healthy(*red))
            return fail(ctx, LBPF_EUNSTABLE, "health check failed at step " + std::to_string(red->step));
    }
    return LBPF_OK;
}

lbpf_status lbpf_history(lbpf_ctx* ctx, lbpf_reductions* out, int32_t max_records, int32_t* count) {
    if (!ctx || !count || (max_records > 0 && !out)) return fail(ctx, LBPF_EINVAL, "bad argument");
    CHK(hipStreamSynchronize(ctx->stream));
    const int64_t avail = std::min<int64_t>(ctx->hist_count, HIST_CAP);
    const int64_t first = ctx->hist_count - avail;
    const int64_t m = std::min<int64_t>(avail, max_records);
    std::vector<double> buf((size_t)HIST_CAP * RED_STRIDE);
    CHK(hipMemcpy(buf.data(), ctx->hist, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
        const int64_t k = (first + i) % HIST_CAP;
        unpack_record(&buf[(size_t)k * RED_STRIDE], &out[i]);
        if (i > 0) set_tip_vel(&out[i], out[i - 1], ctx->prm);
    }
    *count = (int32_t)m;
    return LBPF_OK;
}

lbpf_status lbpf_read_populations(lbpf_ctx* ctx, int32_t field, void* dst) {
    if (!ctx) return LBPF_EINVAL;
    if (field < 0 || field > 2 || !dst) return fail(ctx, LBPF_EINVAL, "bad field or NULL dst");
    CHK(hipStreamSynchronize(ctx->stream));
    const size_t arr = ctx->n * ctx->sbytes, w = ctx->grid.nx * ctx->sbytes, pw = ctx->px * ctx->sbytes;
    const size_t rows = (size_t)ctx->grid.ny * ctx->grid.nz;
    const int es = pop_stride(ctx, field), lane = pop_lane(ctx, field);
    const char* base = (const char*)pop_alloc(ctx, field, ctx->cur);
    std::vector<char> tmp(ctx->na * ctx->sbytes), pairs(es > 1 ? ctx->na * ctx->sbytes * es : 0);
    for (int i = 0; i < lattice_of(ctx, field); ++i) {
        if (es == 1) {
            CHK(hipMemcpy(tmp.data(), base + i * ctx->np * ctx->sbytes, tmp.size(), hipMemcpyDeviceToHost));
        } else {   // this field's elements of the pair array
            CHK(hipMemcpy(pairs.data(), base + i * ctx->np * es * ctx->sbytes, pairs.size(), hipMemcpyDeviceToHost));
            for (size_t k = 0; k < ctx->na; ++k)
                std::memcpy(tmp.data() + k * ctx->sbytes, pairs.data() + (k * es + lane) * ctx->sbytes, ctx->sbytes);
        }
        unpack_rows((char*)dst + i * arr, tmp.data(), w, pw, rows);
    }
    return LBPF_OK;
}

lbpf_status lbpf_write_populations(lbpf_ctx* ctx, int32_t field, const void* src) {
    if (!ctx) return LBPF_EINVAL;
    if (field < 0 || field > 2 || !src) return fail(ctx, LBPF_EINVAL, "bad field or NULL src");
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    CHK(hipStreamSynchronize(ctx->stream));
    const size_t arr = ctx->n * ctx->sbytes, w = ctx->grid.nx * ctx->sbytes, pw = ctx->px * ctx->sbytes;
    const size_t rows = (size_t)ctx->grid.ny * ctx->grid.nz;
    const int es = pop_stride(ctx, field), lane = pop_lane(ctx, field);
    char* base = (char*)pop_alloc(ctx, field, ctx->cur);
    std::vector<char> tmp(ctx->na * ctx->sbytes, 0), pairs(es > 1 ? ctx->na * ctx->sbytes * es : 0);
    for (int i = 0; i < lattice_of(ctx, field); ++i) {
        pack_rows(tmp.data(), (const char*)src + i * arr, w, pw, rows);
        if (es == 1) {
            CHK(hipMemcpy(base + i * ctx->np * ctx->sbytes, tmp.data(), tmp.size(), hipMemcpyHostToDevice));
        } else {   // replace this field's elements of the pair array, keep the other's
            char* dev = base + i * ctx->np * es * ctx->sbytes;
            CHK(hipMemcpy(pairs.data(), dev, pairs.size(), hipMemcpyDeviceToHost));
            for (size_t k = 0; k < ctx->na; ++k)
                std::memcpy(pairs.data() + (k * es + lane) * ctx->sbytes, tmp.data() + k * ctx->sbytes, ctx->sbytes);
            CHK(hipMemcpy(dev, pairs.data(), pairs.size(), hipMemcpyHostToDevice));
        }
    }
    return LBPF_OK;
}

lbpf_status lbpf_read_populations_f64(lbpf_ctx* ctx, int32_t field, double* dst) {
    if (!ctx) return LBPF_EINVAL;
    if (field < 0 || field > 2 || !dst) return fail(ctx, LBPF_EINVAL, "bad field or NULL dst");
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    double* d = nullptr;
    const size_t bytes = ctx->n * lattice_of(ctx, field) * sizeof(double);
    CHK(hipStreamSynchronize(ctx->stream));
    CHK(hipMalloc((void**)&d, bytes));
    lbpf_status st = init_or_decode(ctx, 1, field, d);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (!st && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return fail(ctx, LBPF_EDEVICE, std::string("decode copy: ") + hipGetErrorString(e));
    return LBPF_OK;
}

lbpf_status lbpf_debug_stream_only(lbpf_ctx* ctx, int64_t nsteps) {
    if (!ctx) return LBPF_EINVAL;
    if (nsteps < 0) return fail(ctx, LBPF_EINVAL, "nsteps < 0");
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    for (int64_t s = 0; s < nsteps; ++s) {
        lbpf_status st = stream_only_q(ctx, ctx->q, 0, 1);
        if (!st) st = stream_only_q(ctx, ctx->q_ut, 1, 3);
        if (!st) st = stream_only_fields(ctx);
        if (st) return st;
    }
    return LBPF_OK;
}

lbpf_status lbpf_set_timing(lbpf_ctx* ctx, int32_t enable) {
    if (!ctx) return LBPF_EINVAL;
    const lbpf_status st = drain_launches(ctx, nullptr, nullptr);
    if (st) return st;
    for (int i = 0; i < 3; ++i) { ctx->t_ms[i] = 0; ctx->t_n[i] = 0; }
    ctx->timing = enable != 0;
    return LBPF_OK;
}

lbpf_status lbpf_kernel_times(lbpf_ctx* ctx, double ms[3], int64_t launches[3]) {
    if (!ctx || !ms || !launches) return fail(ctx, LBPF_EINVAL, "bad argument");
    const lbpf_status st = drain_launches(ctx, ctx->t_ms, ctx->t_n);
    if (st) return st;
    for (int i = 0; i < 3; ++i) { ms[i] = ctx->t_ms[i]; launches[i] = ctx->t_n[i]; }
    return LBPF_OK;
}

lbpf_status lbpf_set_kernel_launch(lbpf_ctx* ctx, int32_t kernel, int32_t tile_x, int32_t tile_y,
                                   int32_t zslab, int32_t xcd_remap) {
    if (!ctx) return LBPF_EINVAL;
    if (kernel != K_PHI && kernel != K_UT) return fail(ctx, LBPF_EINVAL, "kernel must be 0 (k_phi) or 1 (k_ut)");
    if (zslab < 1) return fail(ctx, LBPF_EINVAL, "zslab < 1");
    if (xcd_remap != 0 && xcd_remap != 1) return fail(ctx, LBPF_EINVAL, "xcd_remap must be 0 or 1");
    for (int i = 0; i < kNumShapes; ++i) {
        if (kShapes[i].tx != tile_x || kShapes[i].ty != tile_y) continue;
        if (!shape_ok(ctx->storage, i)) return fail(ctx, LBPF_EINVAL, "tile shape not available for this storage");
        if (kernel == K_UT && ut_pinned(ctx) && i != adv_shape(ctx))
            return fail(ctx, LBPF_EINVAL, kAdvTileMsg);
        ctx->shape[kernel] = i;
        ctx->zslab[kernel] = zslab;
        ctx->remap[kernel] = xcd_remap;
        return LBPF_OK;
    }
    return fail(ctx, LBPF_EINVAL, "unsupported tile shape");
}

lbpf_status lbpf_get_kernel_launch(lbpf_ctx* ctx, int32_t kernel, int32_t* tile_x, int32_t* tile_y,
                                   int32_t* zslab, int32_t* xcd_remap) {
    if (!ctx || !tile_x || !tile_y || !zslab || !xcd_remap) return LBPF_EINVAL;
    if (kernel != K_PHI && kernel != K_UT) return fail(ctx, LBPF_EINVAL, "kernel must be 0 (k_phi) or 1 (k_ut)");
    *tile_x = kShapes[ctx->shape[kernel]].tx;
    *tile_y = kShapes[ctx->shape[kernel]].ty;
    *zslab = ctx->zslab[kernel];
    *xcd_remap = ctx->remap[kernel];
    return LBPF_OK;
}

lbpf_status lbpf_set_launch(lbpf_ctx* ctx, int32_t tile_x, int32_t tile_y, int32_t zslab,
                            int32_t xcd_remap) {
    if (!ctx) return LBPF_EINVAL;
    const int s0[2] = {ctx->shape[0], ctx->shape[1]}, z0[2] = {ctx->zslab[0], ctx->zslab[1]},
              r0[2] = {ctx->remap[0], ctx->remap[1]};
    for (int k = 0; k < 2; ++k) {
        const lbpf_status st = lbpf_set_kernel_launch(ctx, k, tile_x, tile_y, zslab, xcd_remap);
        if (st) {   // all or nothing
            for (int j = 0; j < 2; ++j) { ctx->shape[j] = s0[j]; ctx->zslab[j] = z0[j]; ctx->remap[j] = r0[j]; }
            return st;
        }
    }
    return LBPF_OK;
}

lbpf_status lbpf_get_launch(lbpf_ctx* ctx, int32_t* tile_x, int32_t* tile_y, int32_t* zslab,
                            int32_t* xcd_remap) {
    return lbpf_get_kernel_launch(ctx, K_UT, tile_x, tile_y, zslab, xcd_remap);
}

lbpf_status lbpf_autotune(lbpf_ctx* ctx, int32_t steps_per_candidate, double* best_ms_per_step) {
    const lbpf::Range range("lbpf_autotune");
    if (!ctx) return LBPF_EINVAL;
    if (steps_per_candidate < 1) return fail(ctx, LBPF_EINVAL, "steps_per_candidate < 1");
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    CHK(hipStreamSynchronize(ctx->stream));
    // snapshot of the current state (populations and fields of parity cur):
    // the population allocations one after another, then the three fields
    const size_t fbytes = ctx->na * ctx->tbytes;
    size_t pset[3], poff[3], ptot = 0;
    for (int f = 0; f < 3; ++f) {
        pset[f] = pop_alloc_bytes(ctx, f);
        poff[f] = ptot;
        ptot += pset[f];
    }
    void* snap = nullptr;
    CHK(hipMalloc(&snap, ptot + 3 * fbytes));
    const int cur0 = ctx->cur;
    for (int f = 0; f < 3; ++f) {
        if (pset[f])
            CHK(hipMemcpyAsync((char*)snap + poff[f], ctx->pop[f][cur0], pset[f], hipMemcpyDeviceToDevice,
                               ctx->stream));
        CHK(hipMemcpyAsync((char*)snap + ptot + f * fbytes, ctx->fld[f][cur0], fbytes,
                           hipMemcpyDeviceToDevice, ctx->stream));
    }
    // launches timed so far count for the caller; the tuner's own stay apart
    lbpf_status st = drain_launches(ctx, ctx->t_ms, ctx->t_n);
    if (st) { (void)hipFree(snap); return st; }
    const bool was_timing = ctx->timing;
    ctx->timing = true;
    const int s0[2] = {ctx->shape[0], ctx->shape[1]}, z0[2] = {ctx->zslab[0], ctx->zslab[1]},
              r0[2] = {ctx->remap[0], ctx->remap[1]};
    int bs[2] = {s0[0], s0[1]}, bz[2] = {z0[0], z0[1]}, br[2] = {r0[0], r0[1]};
    double best[2] = {1e300, 1e300};
    // k_phi and k_ut are separate launches: each keeps the launch that is
    // fastest for it
    const int zs_list[] = {2, 4, 6, 8, 12, 16};
    constexpr int NZ = sizeof(zs_list) / sizeof(zs_list[0]);
    for (int sh = 0; sh < kNumShapes && !st; ++sh) {
        if (!shape_ok(ctx->storage, sh)) continue;
        for (int zi = 0; zi < 2 * NZ && !st; ++zi) {
            const int zsl = zs_list[zi % NZ];
            if (zsl > 2 * ctx->grid.nz && zi % NZ > 0) continue;
            for (int k = 0; k < 2; ++k) {
                ctx->shape[k] = sh;
                ctx->zslab[k] = zsl;
                ctx->remap[k] = zi / NZ;
            }
            if (ut_pinned(ctx)) ctx->shape[K_UT] = adv_shape(ctx);
            for (int w = 0; w < 2 && !st; ++w) st = launch_step(ctx);
            if (!st) st = drain_launches(ctx, nullptr, nullptr);
            for (int k = 0; k < steps_per_candidate && !st; ++k) st = launch_step(ctx);
            double ms[3] = {0, 0, 0};
            int64_t cnt[3] = {0, 0, 0};
            if (!st) st = drain_launches(ctx, ms, cnt);
            if (st) break;
            for (int k = 0; k < 2; ++k) {
                const double per = ms[k] / steps_per_candidate;
                if (per < best[k]) {
                    best[k] = per;
                    bs[k] = ctx->shape[k];
                    bz[k] = zsl;
                    br[k] = ctx->remap[k];
                }
            }
        }
    }
    // restore the state and keep the best launch of each kernel
    ctx->cur = cur0;
    for (int f = 0; f < 3; ++f) {
        if (pset[f])
            (void)hipMemcpyAsync(ctx->pop[f][cur0], (char*)snap + poff[f], pset[f], hipMemcpyDeviceToDevice,
                                 ctx->stream);
        (void)hipMemcpyAsync(ctx->fld[f][cur0], (char*)snap + ptot + f * fbytes, fbytes,
                             hipMemcpyDeviceToDevice, ctx->stream);
    }
    (void)drain_launches(ctx, nullptr, nullptr);
    (void)hipFree(snap);
    ctx->timing = was_timing;
    const int* keep_s = st ? s0 : bs;
    const int* keep_z = st ? z0 : bz;
    const int* keep_r = st ? r0 : br;
    for (int k = 0; k < 2; ++k) {
        ctx->shape[k] = keep_s[k];
        ctx->zslab[k] = keep_z[k];
        ctx->remap[k] = keep_r[k];
    }
    if (st) return st;
    if (best_ms_per_step) *best_ms_per_step = best[0] + best[1];
    return LBPF_OK;
}

lbpf_status lbpf_autotune_cached(lbpf_ctx* ctx, int32_t steps_per_candidate, const char* cache_path,
                                 int32_t* hit, double* best_ms_per_step) {
    const lbpf::Range range("lbpf_autotune_cached");
    if (!ctx) return LBPF_EINVAL;
    if (!cache_path) return fail(ctx, LBPF_EINVAL, "cache_path is NULL");
    if (hit) *hit = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    CHK(hipGetDevice(&dev));
    CHK(hipGetDeviceProperties(&prop, dev));
    char arch[sizeof(prop.gcnArchName) + 1];
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* a = arch; *a; ++a)
        if (*a == ' ' || *a == '\t') *a = '_';
    char key[512];
    std::snprintf(key, sizeof(key), "lbpf-autotune-2 k%s %s cu%d q%d qut%d s%d %dx%dx%d pin%d", LBPF_KERNEL_BUILD,
                  arch, prop.multiProcessorCount, ctx->q, ctx->q_ut, ctx->storage, ctx->grid.nx, ctx->grid.ny,
                  ctx->grid.nz, ut_pinned(ctx) ? 1 : 0);
    const size_t klen = std::strlen(key);
    if (FILE* in = std::fopen(cache_path, "r")) {
        char line[1024];
        bool found = false;
        while (!found && std::fgets(line, sizeof(line), in)) {
            if (std::strncmp(line, key, klen) != 0 || (line[klen] != ' ' && line[klen] != '\t')) continue;
            int l[2][4];
            double ms = 0.0;
            if (std::sscanf(line + klen, "%d %d %d %d %d %d %d %d %lf", &l[0][0], &l[0][1], &l[0][2], &l[0][3],
                            &l[1][0], &l[1][1], &l[1][2], &l[1][3], &ms) != 9)
                continue;
            // all or nothing: a launch this context refuses leaves the old ones
            const int s0[2] = {ctx->shape[0], ctx->shape[1]}, z0[2] = {ctx->zslab[0], ctx->zslab[1]},
                      r0[2] = {ctx->remap[0], ctx->remap[1]};
            lbpf_status st = LBPF_OK;
            for (int k = 0; k < 2 && !st; ++k)
                st = lbpf_set_kernel_launch(ctx, k, l[k][0], l[k][1], l[k][2], l[k][3]);
            if (st) {
                for (int k = 0; k < 2; ++k) { ctx->shape[k] = s0[k]; ctx->zslab[k] = z0[k]; ctx->remap[k] = r0[k]; }
                ctx->err.clear();
                continue;
            }
            found = true;
            if (hit) *hit = 1;
            if (best_ms_per_step) *best_ms_per_step = ms;
        }
        const bool bad = std::ferror(in) != 0;
        std::fclose(in);
        if (found) return LBPF_OK;
        if (bad) return fail(ctx, LBPF_EIO, std::string("cannot read ") + cache_path);
    }
    double best = 0.0;
    const lbpf_status st = lbpf_autotune(ctx, steps_per_candidate, &best);
    if (st) return st;
    if (best_ms_per_step) *best_ms_per_step = best;
    char line[1024];
    int n = std::snprintf(line, sizeof(line), "%s", key);
    for (int k = 0; k < 2; ++k) {
        const Shape sh = kShapes[ctx->shape[k]];
        n += std::snprintf(line + n, sizeof(line) - n, " %d %d %d %d", sh.tx, sh.ty, ctx->zslab[k], ctx->remap[k]);
    }
    std::snprintf(line + n, sizeof(line) - n, " %.6f\n", best);
    FILE* out = std::fopen(cache_path, "a");
    if (!out) return fail(ctx, LBPF_EIO, std::string("cannot append to ") + cache_path);
    const bool ok = std::fputs(line, out) >= 0;
    const bool closed = std::fclose(out) == 0;
    if (!ok || !closed) return fail(ctx, LBPF_EIO, std::string("cannot append to ") + cache_path);
    return LBPF_OK;
}

// Device-resident field I/O: convert between the caller's FP32/FP64 arrays
// and the context's field type on the context's stream.
// in_pitched / out_pitched: the array has the context's row pitch (its own
// fields), else rows of nx (the caller's arrays).
lbpf_status convert_field(lbpf_ctx* ctx, const void* in, int32_t in_f64, bool in_pitched, void* out,
                          int32_t out_f64, bool out_pitched) {
    const int nx = ctx->grid.nx;
    const size_t rows = (size_t)ctx->grid.ny * ctx->grid.nz;
    const int pin = in_pitched ? ctx->px : nx, pout = out_pitched ? ctx->px : nx;
    const int nb = (int)std::min<size_t>(8192, (ctx->n + 255) / 256);
    if (in_f64 && out_f64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(nb), dim3(256), 0, ctx->stream, (const double*)in,
                           (double*)out, nx, pin, pout, rows);
    else if (in_f64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(256), 0, ctx->stream, (const double*)in,
                           (float*)out, nx, pin, pout, rows);
    else if (out_f64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, ctx->stream, (const float*)in,
                           (double*)out, nx, pin, pout, rows);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(nb), dim3(256), 0, ctx->stream, (const float*)in,
                           (float*)out, nx, pin, pout, rows);
    CHK(hipGetLastError());
    return LBPF_OK;
}

lbpf_status lbpf_set_velocity_field(lbpf_ctx* ctx, const double* vx, const double* vy, const double* vz) {
    if (!ctx) return LBPF_EINVAL;
    if (ctx->in_batch) return fail(ctx, LBPF_ESTATE, "batched domains have no advective velocity");
    if (ctx->prm.skip_theta && (vx || vy || vz))
        return fail(ctx, LBPF_EINVAL, "advection needs the heat equation (skip_theta = 0)");
    const size_t n = ctx->n;
    if (!vx && !vy && !vz) {
        CHK(hipStreamSynchronize(ctx->stream));
        if (ctx->vfield) CHK(hipFree(ctx->vfield));
        ctx->vfield = nullptr;
    } else {
        if (!vx || !vy || !vz) return fail(ctx, LBPF_EINVAL, "give all three velocity components or none");
        const double scale = ctx->prm.dt / (lattice_e2(ctx->q_ut) * ctx->prm.dx);   // theta's lattice
        // device layout: three arrays of na values with the fields' row pitch
        const size_t na = ctx->na, nx = ctx->grid.nx;
        std::vector<char> host(3 * na * ctx->tbytes, 0);
        const double* comp[3] = {vx, vy, vz};
        for (int a = 0; a < 3; ++a)
            for (size_t i = 0; i < n; ++i) {
                const double v = comp[a][i];
                if (!std::isfinite(v)) return fail(ctx, LBPF_EINVAL, "advective velocity must be finite");
                const size_t d = a * na + (i / nx) * ctx->px + i % nx;
                if (ctx->tbytes == 8) ((double*)host.data())[d] = v * scale;
                else ((float*)host.data())[d] = (float)(v * scale);
            }
        CHK(hipStreamSynchronize(ctx->stream));
        if (!ctx->vfield && hipMalloc(&ctx->vfield, host.size()) != hipSuccess) {
            ctx->vfield = nullptr;
            return fail(ctx, LBPF_ENOMEM, "hipMalloc of the velocity field failed");
        }
        CHK(hipMemcpy(ctx->vfield, host.data(), host.size(), hipMemcpyHostToDevice));
        // the advective variant of k_ut exists for one tile
        ctx->shape[K_UT] = adv_shape(ctx);
    }
    // a captured step loop holds the old constants
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    return LBPF_OK;
}

lbpf_status lbpf_set_fields_device(lbpf_ctx* ctx, const void* phi, const void* U, const void* theta,
                                   int32_t dtype) {
    if (!ctx) return LBPF_EINVAL;
    if (!phi || !U || !theta) return fail(ctx, LBPF_EINVAL, "NULL field array");
    if (dtype != LBPF_FIELD_F32 && dtype != LBPF_FIELD_F64) return fail(ctx, LBPF_EINVAL, "dtype must be 0 or 1");
    ctx->cur = 0;
    const void* src[3] = {phi, U, theta};
    for (int f = 0; f < 3; ++f) {
        lbpf_status st = convert_field(ctx, src[f], dtype == LBPF_FIELD_F64, false, ctx->fld[f][0],
                                       ctx->tbytes == 8, true);
        if (st) return st;
    }
    lbpf_status st = init_or_decode(ctx, 0, 0, nullptr);
    if (st) return st;
    CHK(hipStreamSynchronize(ctx->stream));
    ctx->have_fields = true;
    ctx->step = 0;
    ctx->hist_count = 0;
    return LBPF_OK;
}

lbpf_status lbpf_read_fields_device(lbpf_ctx* ctx, void* phi, void* U, void* theta, int32_t dtype) {
    if (!ctx) return LBPF_EINVAL;
    if (!ctx->have_fields) return fail(ctx, LBPF_ESTATE, "lbpf_set_fields has not been called");
    if (dtype != LBPF_FIELD_F32 && dtype != LBPF_FIELD_F64) return fail(ctx, LBPF_EINVAL, "dtype must be 0 or 1");
    void* dst[3] = {phi, U, theta};
    for (int f = 0; f < 3; ++f) {
        if (!dst[f]) continue;
        lbpf_status st = convert_field(ctx, ctx->fld[f][ctx->cur], ctx->tbytes == 8, true, dst[f],
                                       dtype == LBPF_FIELD_F64, false);
        if (st) return st;
    }
    return LBPF_OK;
}

lbpf_status lbpf_bench_bandwidth(int32_t mode, int32_t width, int32_t nontemporal, int32_t blocks, void* dst,
                                 const void* src, int64_t nbytes, void* hip_stream) {
    if (mode < 0 || mode > 2 || (width != 2 && width != 4 && width != 8 && width != 16) || blocks < 0 || nbytes < 0 ||
        (nbytes % width) != 0 || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16) ||
        (mode != 1 && !src) || !dst)
        return LBPF_EINVAL;
    const size_t n = (size_t)nbytes / width;
    if (n == 0) return LBPF_OK;
    // default grid: one thread per four elements, capped at 2^20 threads
    const int nb = blocks ? blocks : (int)std::min<size_t>(4096, (n / 4 + 255) / 256 + 1);
    const hipStream_t st = (hipStream_t)hip_stream;
    if (width == 2) launch_bw_mode<unsigned short>(mode, nontemporal, nb, st, src, dst, n);
    else if (width == 4) launch_bw_mode<unsigned>(mode, nontemporal, nb, st, src, dst, n);
    else if (width == 8) launch_bw_mode<u32x2>(mode, nontemporal, nb, st, src, dst, n);
    else launch_bw_mode<u32x4>(mode, nontemporal, nb, st, src, dst, n);
    return hipGetLastError() == hipSuccess ? LBPF_OK : LBPF_EDEVICE;
}

lbpf_status lbpf_reduce_fields_noalloc(const void* phi, const void* U, const void* theta, int32_t dtype,
                                       int32_t nx, int32_t ny, int32_t nz, double k, double dx,
                                       const double* centre, double* rec, void* hip_stream) {
    if (!phi || !U || !theta || !centre || !rec)
        return fail(nullptr, LBPF_EINVAL, "lbpf_reduce_fields_noalloc: NULL argument");
    if (dtype != LBPF_FIELD_F32 && dtype != LBPF_FIELD_F64)
        return fail(nullptr, LBPF_EINVAL, "lbpf_reduce_fields_noalloc: dtype must be 0 (FP32) or 1 (FP64)");
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(nullptr, LBPF_EINVAL, "lbpf_reduce_fields_noalloc: nx, ny, nz must be >= 1");
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    if (n > kNoallocMaxNodes)
        return fail(nullptr, LBPF_EINVAL,
                    "lbpf_reduce_fields_noalloc: more than 2^31 nodes (the limit of this entry point)");
    if (!(k > 0.0 && k < 1.0) || !(dx > 0.0))
        return fail(nullptr, LBPF_EINVAL, "lbpf_reduce_fields_noalloc: k must lie in (0,1) and dx be > 0");
    void* part = nullptr;
    hipError_t e = scratch_on_device(&part);
    if (e != hipSuccess)
        return fail(nullptr, LBPF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    const hipStream_t st = (hipStream_t)hip_stream;
    // same grid as the context reductions: results equal theirs bit for bit
    const int nb = (int)std::min<size_t>(RED_BLOCKS_NOALLOC, (n + 255) / 256);
    if (dtype == LBPF_FIELD_F64)
        hipLaunchKernelGGL((k_reduce_part<double>), dim3(nb), dim3(256), 0, st, nx, ny, nz, nx, k, dx * dx * dx,
                           (const double*)phi, (const double*)U, (const double*)theta, (double*)part);
    else
        hipLaunchKernelGGL((k_reduce_part<float>), dim3(nb), dim3(256), 0, st, nx, ny, nz, nx, k, dx * dx * dx,
                           (const float*)phi, (const float*)U, (const float*)theta, (double*)part);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, (const double*)part, nb, 1.0 / (double)n,
                           centre[0], centre[1], centre[2], 0LL, rec);
        e = hipGetLastError();
    }
    if (e != hipSuccess)
        return fail(nullptr, LBPF_EDEVICE, std::string("lbpf_reduce_fields_noalloc: ") + hipGetErrorString(e));
    return LBPF_OK;
}

lbpf_status lbpf_bench_copy(void* dst, const void* src, int64_t nbytes, void* hip_stream) {
    if (!dst || !src || nbytes < 0 || (nbytes % 16) != 0 || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return LBPF_EINVAL;
    const int nb = (int)std::min<int64_t>(32768, (nbytes / 16 + 255) / 256);
    return lbpf_bench_bandwidth(2, 16, 1, nb > 0 ? nb : 1, dst, src, nbytes, hip_stream);
}

}  // extern "C"

// ---------------------------------------------------------------- batches
namespace {

#define BCHK(call)                                                                 \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            b->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
            return LBPF_EDEVICE;                                                   \
        }                                                                          \
    } while (0)

lbpf_status bfail(lbpf_batch* b, lbpf_status s, const std::string& m) {
    if (b) b->err = m;
    else g_create_error = m;
    return s;
}

template <class T>
lbpf_status batch_build_t(lbpf_batch* b) {
    const int nd = (int)b->dom.size();
    std::vector<DomainDesc<T>> desc(nd);
    std::vector<int2> items[2][3];
    for (int d = 0; d < nd; ++d) {
        lbpf_ctx* c = b->dom[d];
        for (int k = 0; k < 2; ++k) {
            c->shape[k] = b->shape[k];
            c->zslab[k] = b->zslab[k];
            c->remap[k] = 0;   // the work table carries the XCD order
        }
        for (int k = 0; k < 2; ++k) desc[d].c[k] = make_coef<T>(c, k);
        for (int f = 0; f < 3; ++f)
            for (int par = 0; par < 2; ++par) {
                desc[d].pop[f][par] = c->pop[f][par];
                desc[d].fld[f][par] = (T*)c->fld[f][par];
            }
        for (int k = 0; k < 2; ++k) {
            const int q = k == K_PHI ? c->q : c->q_ut;
            const int li = q == 7 ? 0 : q == 15 ? 1 : 2;
            const int nt = total_tiles(c, k);
            for (int t = 0; t < nt; ++t) items[k][li].push_back(int2{d, t});
        }
    }
    if (!b->d_desc) BCHK(hipMalloc(&b->d_desc, sizeof(DomainDesc<T>) * nd));
    BCHK(hipMemcpy(b->d_desc, desc.data(), sizeof(DomainDesc<T>) * nd, hipMemcpyHostToDevice));
    for (int kl = 0; kl < 6; ++kl) {
        const int k = kl / 3, li = kl % 3;
        std::vector<int2>& it = items[k][li];
        if (b->d_work[k][li]) { (void)hipFree(b->d_work[k][li]); b->d_work[k][li] = nullptr; }
        b->nwork[k][li] = 0;
        if (it.empty()) continue;
        while (it.size() % 8) it.push_back(int2{-1, 0});
        // block k*8 + x runs on XCD x: give each XCD a contiguous run of tiles
        const size_t m = it.size() / 8;
        std::vector<int2> w(it.size());
        for (size_t blk = 0; blk < it.size(); ++blk) w[blk] = it[(blk % 8) * m + blk / 8];
        BCHK(hipMalloc((void**)&b->d_work[k][li], sizeof(int2) * w.size()));
        BCHK(hipMemcpy(b->d_work[k][li], w.data(), sizeof(int2) * w.size(), hipMemcpyHostToDevice));
        b->nwork[k][li] = (int)w.size();
    }
    b->built = true;
    return LBPF_OK;
}

template <class T, class S>
hipError_t batch_launch_ts(lbpf_batch* b, int k, int li, int par) {
    const int2* w = b->d_work[k][li];
    const int n = b->nwork[k][li];
    switch (li) {
        case 0: return batch_launch_s<D3Q7, T, S>(k, b->shape[k], b->d_desc, w, n, par, b->stream);
        case 1: return batch_launch_s<D3Q15, T, S>(k, b->shape[k], b->d_desc, w, n, par, b->stream);
        default: return batch_launch_s<D3Q19, T, S>(k, b->shape[k], b->d_desc, w, n, par, b->stream);
    }
}

// Launches of kernel k (K_PHI or K_UT) for every lattice present in the batch.
lbpf_status batch_launch_kernel(lbpf_batch* b, int k, int par) {
    for (int li = 0; li < 3; ++li) {
        if (!b->nwork[k][li]) continue;
        hipError_t e = hipErrorInvalidValue;
        switch (b->storage) {
            case LBPF_F32: e = batch_launch_ts<float, float>(b, k, li, par); break;
            case LBPF_F16_DEV: e = batch_launch_ts<float, __half>(b, k, li, par); break;
            case LBPF_BF16_DEV: e = batch_launch_ts<float, __hip_bfloat16>(b, k, li, par); break;
            case LBPF_F64: e = batch_launch_ts<double, double>(b, k, li, par); break;
        }
        if (e != hipSuccess) return bfail(b, LBPF_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    }
    return LBPF_OK;
}

// One time step of every domain: phase field of all domains, then U/theta.
lbpf_status batch_step_once(lbpf_batch* b, int par) {
    lbpf_status st = batch_launch_kernel(b, K_PHI, par);
    if (!st) st = batch_launch_kernel(b, K_UT, par);
    return st;
}

lbpf_status batch_build(lbpf_batch* b) {
    if (b->gexec) {   // a captured graph holds the old work tables
        (void)hipStreamSynchronize(b->stream);
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return b->storage == LBPF_F64 ? batch_build_t<double>(b) : batch_build_t<float>(b);
}

}  // namespace

extern "C" {

lbpf_status lbpf_batch_create(int32_t n, const lbpf_grid* grids, const lbpf_params* params,
                              void* hip_stream, lbpf_batch** out) {
    if (!out) return bfail(nullptr, LBPF_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !grids || !params) return bfail(nullptr, LBPF_EINVAL, "need n >= 1 grids and params");
    for (int i = 1; i < n; ++i)
        if (grids[i].storage != grids[0].storage)
            return bfail(nullptr, LBPF_EINVAL, "all domains of a batch share one storage type");
    for (int i = 0; i < n; ++i) {
        if (grids[i].lattice != LBPF_D3Q7 && grids[i].lattice != LBPF_D3Q15 && grids[i].lattice != LBPF_D3Q19)
            return bfail(nullptr, LBPF_EINVAL, "batched domains use D3Q7, D3Q15 or D3Q19");
        if (grids[i].lattice_ut != 0 && grids[i].lattice_ut != LBPF_D3Q7 && grids[i].lattice_ut != LBPF_D3Q15 &&
            grids[i].lattice_ut != LBPF_D3Q19)
            return bfail(nullptr, LBPF_EINVAL, "lattice_ut must be 0, 7, 15 or 19");
        if (params[i].vel[0] != 0.0 || params[i].vel[1] != 0.0 || params[i].vel[2] != 0.0)
            return bfail(nullptr, LBPF_EINVAL, "batched domains have no advective velocity");
        if (params[i].skip_U || params[i].skip_theta)
            return bfail(nullptr, LBPF_EINVAL, "batched domains solve U and theta");
    }
    lbpf_batch* b = new (std::nothrow) lbpf_batch();
    if (!b) return bfail(nullptr, LBPF_ENOMEM, "host allocation failed");
    b->storage = grids[0].storage;
    for (int k = 0; k < 2; ++k) {   // defaults measured for the batch kernels
        b->shape[k] = b->storage == LBPF_F64 ? 2 : 3;   // 32x4 (FP64) or 32x8 tiles
        b->zslab[k] = lbpf_storage_bytes(b->storage) == 2 ? 8 : 4;
    }
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return bfail(nullptr, LBPF_EDEVICE, "hipStreamCreateWithFlags failed");
        }
        b->own_stream = true;
    }
    for (int i = 0; i < n; ++i) {
        lbpf_ctx* c = nullptr;
        const lbpf_status st = lbpf_create(&grids[i], &params[i], b->stream, &c);
        if (st) {
            const std::string msg = "domain " + std::to_string(i) + ": " + g_create_error;
            for (lbpf_ctx* d : b->dom) lbpf_destroy(d);
            if (b->own_stream) (void)hipStreamDestroy(b->stream);
            delete b;
            return bfail(nullptr, st, msg);
        }
        c->in_batch = true;
        b->dom.push_back(c);
        if (std::max(pop_alloc_bytes(c, 0), pop_alloc_bytes(c, 1)) >= ((size_t)1 << 32) - 256) {
            for (lbpf_ctx* d : b->dom) { d->in_batch = false; lbpf_destroy(d); }
            if (b->own_stream) (void)hipStreamDestroy(b->stream);
            delete b;
            return bfail(nullptr, LBPF_EINVAL, "batch domains must hold < 4 GiB of populations per field");
        }
    }
    *out = b;
    return LBPF_OK;
}

lbpf_ctx* lbpf_batch_domain(lbpf_batch* b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->dom.size()) return nullptr;
    return b->dom[i];
}

lbpf_status lbpf_batch_set_graph(lbpf_batch* b, int32_t steps_per_graph) {
    if (!b) return LBPF_EINVAL;
    if (steps_per_graph < 0 || (steps_per_graph % 2) != 0)
        return bfail(b, LBPF_EINVAL, "steps_per_graph must be 0 or a positive even number");
    b->graph_steps = steps_per_graph;
    if (b->gexec) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return LBPF_OK;
}

lbpf_status lbpf_batch_set_launch(lbpf_batch* b, int32_t kernel, int32_t tile_x, int32_t tile_y, int32_t zslab) {
    if (!b) return LBPF_EINVAL;
    if (kernel != K_PHI && kernel != K_UT) return bfail(b, LBPF_EINVAL, "kernel must be 0 (k_phi) or 1 (k_ut)");
    if (zslab < 1) return bfail(b, LBPF_EINVAL, "zslab < 1");
    for (int i = 0; i < kNumShapes; ++i) {
        if (kShapes[i].tx != tile_x || kShapes[i].ty != tile_y) continue;
        if (!shape_ok(b->storage, i)) return bfail(b, LBPF_EINVAL, "tile shape not available for this storage");
        b->shape[kernel] = i;
        b->zslab[kernel] = zslab;
        b->built = false;
        return LBPF_OK;
    }
    return bfail(b, LBPF_EINVAL, "unsupported tile shape");
}

lbpf_status lbpf_batch_get_launch(lbpf_batch* b, int32_t kernel, int32_t* tile_x, int32_t* tile_y,
                                  int32_t* zslab) {
    if (!b || !tile_x || !tile_y || !zslab) return LBPF_EINVAL;
    if (kernel != K_PHI && kernel != K_UT) return bfail(b, LBPF_EINVAL, "kernel must be 0 (k_phi) or 1 (k_ut)");
    *tile_x = kShapes[b->shape[kernel]].tx;
    *tile_y = kShapes[b->shape[kernel]].ty;
    *zslab = b->zslab[kernel];
    return LBPF_OK;
}

lbpf_status lbpf_batch_autotune(lbpf_batch* b, int32_t steps_per_candidate, double* best_ms_per_step) {
    const lbpf::Range range("lbpf_batch_autotune");
    if (!b) return LBPF_EINVAL;
    if (steps_per_candidate < 1) return bfail(b, LBPF_EINVAL, "steps_per_candidate < 1");
    const int cur0 = b->dom[0]->cur;
    for (lbpf_ctx* c : b->dom) {
        if (!c->have_fields) return bfail(b, LBPF_ESTATE, "a domain has no fields yet");
        if (c->cur != cur0) return bfail(b, LBPF_ESTATE, "domains are at different parities");
    }
    BCHK(hipStreamSynchronize(b->stream));
    // snapshot of every domain's state (populations and fields of parity cur0)
    std::vector<size_t> off;
    size_t total = 0;
    for (lbpf_ctx* c : b->dom) {
        off.push_back(total);
        for (int f = 0; f < 3; ++f) total += pop_alloc_bytes(c, f) + c->na * c->tbytes;
    }
    char* snap = nullptr;
    BCHK(hipMalloc((void**)&snap, total));
    auto copy_state = [&](bool save) -> hipError_t {
        for (size_t d = 0; d < b->dom.size(); ++d) {
            lbpf_ctx* c = b->dom[d];
            size_t o = off[d];
            for (int f = 0; f < 3; ++f) {
                const size_t pb = pop_alloc_bytes(c, f), fb = c->na * c->tbytes;
                hipError_t e = hipSuccess;
                if (pb)
                    e = save ? hipMemcpyAsync(snap + o, c->pop[f][cur0], pb, hipMemcpyDeviceToDevice, b->stream)
                             : hipMemcpyAsync(c->pop[f][cur0], snap + o, pb, hipMemcpyDeviceToDevice, b->stream);
                if (e != hipSuccess) return e;
                o += pb;
                e = save ? hipMemcpyAsync(snap + o, c->fld[f][cur0], fb, hipMemcpyDeviceToDevice, b->stream)
                         : hipMemcpyAsync(c->fld[f][cur0], snap + o, fb, hipMemcpyDeviceToDevice, b->stream);
                if (e != hipSuccess) return e;
                o += fb;
            }
        }
        return hipSuccess;
    };
    hipError_t e = copy_state(true);
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    const int s0[2] = {b->shape[0], b->shape[1]}, z0[2] = {b->zslab[0], b->zslab[1]};
    int bs[2] = {s0[0], s0[1]}, bz[2] = {z0[0], z0[1]};
    double best[2] = {1e300, 1e300};
    lbpf_status st = e == hipSuccess ? LBPF_OK : bfail(b, LBPF_EDEVICE, hipGetErrorString(e));
    const int zs_list[] = {2, 4, 6, 8, 12};
    for (int sh = 0; sh < kNumShapes && !st; ++sh) {
        if (!shape_ok(b->storage, sh)) continue;
        for (int zsl : zs_list) {
            for (int k = 0; k < 2; ++k) { b->shape[k] = sh; b->zslab[k] = zsl; }
            st = batch_build(b);
            int par = cur0;
            for (int w = 0; w < 2 && !st; ++w) { st = batch_step_once(b, par); par = 1 - par; }
            double ms[2] = {0, 0};
            for (int it = 0; it < steps_per_candidate && !st; ++it) {
                if (hipEventRecord(ev[0], b->stream) != hipSuccess) { st = bfail(b, LBPF_EDEVICE, "event"); break; }
                st = batch_launch_kernel(b, K_PHI, par);
                if (!st && hipEventRecord(ev[1], b->stream) != hipSuccess) st = bfail(b, LBPF_EDEVICE, "event");
                if (!st) st = batch_launch_kernel(b, K_UT, par);
                if (!st && hipEventRecord(ev[2], b->stream) != hipSuccess) st = bfail(b, LBPF_EDEVICE, "event");
                if (!st && hipEventSynchronize(ev[2]) != hipSuccess) st = bfail(b, LBPF_EDEVICE, "event sync");
                float a = 0.f, c2 = 0.f;
                if (!st && (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess ||
                            hipEventElapsedTime(&c2, ev[1], ev[2]) != hipSuccess))
                    st = bfail(b, LBPF_EDEVICE, "event time");
                ms[0] += a;
                ms[1] += c2;
                par = 1 - par;
            }
            if (st) break;
            for (int k = 0; k < 2; ++k) {
                const double per = ms[k] / steps_per_candidate;
                if (per < best[k]) { best[k] = per; bs[k] = sh; bz[k] = zsl; }
            }
        }
    }
    // keep the best launch of each kernel and restore the state
    for (int k = 0; k < 2; ++k) {
        b->shape[k] = st ? s0[k] : bs[k];
        b->zslab[k] = st ? z0[k] : bz[k];
    }
    b->built = false;
    (void)hipStreamSynchronize(b->stream);
    const hipError_t er = copy_state(false);
    for (lbpf_ctx* c : b->dom) c->cur = cur0;
    (void)hipStreamSynchronize(b->stream);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(snap);
    if (st) return st;
    if (er != hipSuccess) return bfail(b, LBPF_EDEVICE, std::string("restore: ") + hipGetErrorString(er));
    if (best_ms_per_step) *best_ms_per_step = best[0] + best[1];
    return LBPF_OK;
}

lbpf_status lbpf_batch_step(lbpf_batch* b, int64_t nsteps) {
    const lbpf::Range range("lbpf_batch_step");
    if (!b) return LBPF_EINVAL;
    if (nsteps < 0) return bfail(b, LBPF_EINVAL, "nsteps < 0");
    const int cur = b->dom[0]->cur;
    for (lbpf_ctx* c : b->dom) {
        if (!c->have_fields) return bfail(b, LBPF_ESTATE, "a domain has no fields yet");
        if (c->cur != cur) return bfail(b, LBPF_ESTATE, "domains are at different parities");
    }
    if (!b->built) {
        lbpf_status st = batch_build(b);
        if (st) return st;
    }
    int par = cur;
    int64_t left = nsteps;
    const int G = b->graph_steps;
    while (left > 0) {
        if (G > 0 && left >= G) {
            if (!b->gexec || b->g_cur != par) {
                if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
                hipGraph_t g = nullptr;
                BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                lbpf_status st = LBPF_OK;
                int p = par;
                for (int k = 0; k < G && !st; ++k) { st = batch_step_once(b, p); p = 1 - p; }
                const hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (st) { if (g) (void)hipGraphDestroy(g); return st; }
                if (e != hipSuccess) return bfail(b, LBPF_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
                const hipError_t e2 = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e2 != hipSuccess) { b->gexec = nullptr; return bfail(b, LBPF_EDEVICE, "graph instantiate"); }
                b->g_cur = par;
            }
            BCHK(hipGraphLaunch(b->gexec, b->stream));
            left -= G;
            for (lbpf_ctx* c : b->dom) c->step += G;
        } else {
            lbpf_status st = batch_step_once(b, par);
            if (st) return st;
            par = 1 - par;
            left--;
            for (lbpf_ctx* c : b->dom) { c->cur = par; c->step++; }
        }
    }
    return LBPF_OK;
}

lbpf_status lbpf_batch_sync(lbpf_batch* b) {
    if (!b) return LBPF_EINVAL;
    BCHK(hipStreamSynchronize(b->stream));
    return LBPF_OK;
}

lbpf_status lbpf_batch_destroy(lbpf_batch* b) {
    if (!b) return LBPF_OK;
    (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->d_desc) (void)hipFree(b->d_desc);
    for (int k = 0; k < 2; ++k)
        for (int li = 0; li < 3; ++li)
            if (b->d_work[k][li]) (void)hipFree(b->d_work[k][li]);
    for (lbpf_ctx* c : b->dom) {
        c->in_batch = false;
        lbpf_destroy(c);
    }
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBPF_OK;
}

const char* lbpf_batch_last_error(const lbpf_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
