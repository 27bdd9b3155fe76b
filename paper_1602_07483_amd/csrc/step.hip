// step.hip -- launches of the two step kernels (Sec. 3.4 order: k_phi, then
// k_ut with the new phase field) for one lattice and storage type.  The build
// compiles this file once per pair, with LBPF_STEP_Q (7, 15 or 19) and
// LBPF_STEP_STORAGE (an lbpf_storage value) defined.
#include "runtime.hpp"

#if !defined(LBPF_STEP_Q) || !defined(LBPF_STEP_STORAGE)
#error "compile with -DLBPF_STEP_Q=<7|15|19> -DLBPF_STEP_STORAGE=<0..3>"
#endif

namespace lbpf_rt {
namespace {

template <class L, class T, class S, int TX, int TY, bool BUF>
lbpf_status launch_phi(lbpf_ctx* ctx) {
    const Coef<T> c = make_coef<T>(ctx, K_PHI);
    const int nb = total_tiles(ctx, K_PHI);
    const int a = ctx->cur, b = 1 - ctx->cur;
    return timed(ctx, K_PHI, [&] {
        hipLaunchKernelGGL((k_phi<L, T, S, TX, TY, BUF>), dim3(nb), dim3(TX * TY), 0, ctx->stream, c,
                           (const S*)ctx->pop[0][a], (S*)ctx->pop[0][b], (const T*)ctx->fld[0][a],
                           (const T*)ctx->fld[1][a], (const T*)ctx->fld[2][a], (T*)ctx->fld[0][b]);
    });
}

template <class L, class T, class S, int TX, int TY, bool BUF>
lbpf_status launch_ut(lbpf_ctx* ctx) {
    const Coef<T> c = make_coef<T>(ctx, K_UT);
    const int nb = total_tiles(ctx, K_UT);
    const int a = ctx->cur, b = 1 - ctx->cur;
    // the advection-diffusion, theta-only and U-only variants exist for one tile
    constexpr int kAdv = kAdvShape[LBPF_STEP_STORAGE];
    constexpr bool kAdvTile = TX == kShapes[kAdv].tx && TY == kShapes[kAdv].ty;
    const bool su = ctx->prm.skip_U == 0, sth = ctx->prm.skip_theta == 0;
    if ((c.has_adv || !su || !sth) && !kAdvTile) return fail(ctx, LBPF_EINVAL, kAdvTileMsg);
    return timed(ctx, K_UT, [&] {
        auto args = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(nb), dim3(TX * TY), 0, ctx->stream, c, (const S*)ctx->pop[1][a],
                               (S*)ctx->pop[1][b], (const S*)ctx->pop[2][a], (S*)ctx->pop[2][b],
                               (const T*)ctx->fld[0][a], (const T*)ctx->fld[0][b], (const T*)ctx->fld[1][a],
                               (const T*)ctx->fld[2][a], (T*)ctx->fld[1][b], (T*)ctx->fld[2][b]);
        };
        if constexpr (kAdvTile) {
            if (c.has_adv && su) return args(k_ut<L, T, S, TX, TY, BUF, true, true, true>);
            if (c.has_adv) return args(k_ut<L, T, S, TX, TY, BUF, true, false, true>);
            if (!su) return args(k_ut<L, T, S, TX, TY, BUF, false, false, true>);
            if (!sth) return args(k_ut<L, T, S, TX, TY, BUF, false, true, false>);
        }
        args(k_ut<L, T, S, TX, TY, BUF, false, true, true>);
    });
}

// One buffer resource per population array when it holds < 4 GiB (for k_ut
// the pair array of h and f when they share one).
template <class L, class T, class S, int K, int TX, int TY>
lbpf_status launch_t(lbpf_ctx* ctx) {
    const size_t pbytes = (size_t)L::Q * ctx->np * sizeof(S) * (size_t)(K == K_UT ? ctx->hs : 1);
    const bool buf = pbytes < ((size_t)1 << 32) - 256;
    if constexpr (sizeof(T) == 8) {
        if (!buf) return fail(ctx, LBPF_EINVAL, "FP64 verification build limited to < 4 GiB per field");
        return K == K_PHI ? launch_phi<L, T, S, TX, TY, true>(ctx) : launch_ut<L, T, S, TX, TY, true>(ctx);
    } else {
        if (K == K_PHI)
            return buf ? launch_phi<L, T, S, TX, TY, true>(ctx) : launch_phi<L, T, S, TX, TY, false>(ctx);
        return buf ? launch_ut<L, T, S, TX, TY, true>(ctx) : launch_ut<L, T, S, TX, TY, false>(ctx);
    }
}

template <class L, class T, class S, int K>
lbpf_status launch_k(lbpf_ctx* ctx) {
    if constexpr (sizeof(T) == 8) {
        switch (ctx->shape[K]) {
            case 0: return launch_t<L, T, S, K, 64, 2>(ctx);
            case 2: return launch_t<L, T, S, K, 32, 4>(ctx);
        }
    } else {
        switch (ctx->shape[K]) {
            case 0: return launch_t<L, T, S, K, 64, 2>(ctx);
            case 1: return launch_t<L, T, S, K, 64, 4>(ctx);
            case 2: return launch_t<L, T, S, K, 32, 4>(ctx);
            case 3: return launch_t<L, T, S, K, 32, 8>(ctx);
            case 4: return launch_t<L, T, S, K, 32, 16>(ctx);
        }
    }
    return fail(ctx, LBPF_EINVAL, "tile shape not available for this storage");
}

}  // namespace

template <class L, class T, class S>
lbpf_status launch_step_s(lbpf_ctx* ctx) {
    lbpf_status st = launch_k<L, T, S, K_PHI>(ctx);
    if (st) return st;
    st = launch_k<L, T, S, K_UT>(ctx);
    if (st) return st;
    ctx->cur = 1 - ctx->cur;
    return LBPF_OK;
}

template <class L, class T, class S>
lbpf_status launch_phi_s(lbpf_ctx* ctx) { return launch_k<L, T, S, K_PHI>(ctx); }

namespace {
template <class L, class T, class S, int TX, int TY>
hipError_t batch_launch_t(int kernel, const void* desc, const int2* work, int nwork, int par, hipStream_t st) {
    if (kernel == K_PHI)
        hipLaunchKernelGGL((k_phi_batch<L, T, S, TX, TY>), dim3(nwork), dim3(TX * TY), 0, st,
                           (const DomainDesc<T>*)desc, work, par);
    else
        hipLaunchKernelGGL((k_ut_batch<L, T, S, TX, TY>), dim3(nwork), dim3(TX * TY), 0, st,
                           (const DomainDesc<T>*)desc, work, par);
    return hipGetLastError();
}
}  // namespace

template <class L, class T, class S>
hipError_t batch_launch_s(int kernel, int shape, const void* desc, const int2* work, int nwork, int par,
                          hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        switch (shape) {
            case 0: return batch_launch_t<L, T, S, 64, 2>(kernel, desc, work, nwork, par, st);
            case 2: return batch_launch_t<L, T, S, 32, 4>(kernel, desc, work, nwork, par, st);
        }
    } else {
        switch (shape) {
            case 0: return batch_launch_t<L, T, S, 64, 2>(kernel, desc, work, nwork, par, st);
            case 1: return batch_launch_t<L, T, S, 64, 4>(kernel, desc, work, nwork, par, st);
            case 2: return batch_launch_t<L, T, S, 32, 4>(kernel, desc, work, nwork, par, st);
            case 3: return batch_launch_t<L, T, S, 32, 8>(kernel, desc, work, nwork, par, st);
            case 4: return batch_launch_t<L, T, S, 32, 16>(kernel, desc, work, nwork, par, st);
        }
    }
    return hipErrorInvalidValue;
}

template <class L, class T, class S>
lbpf_status launch_ut_s(lbpf_ctx* ctx) { return launch_k<L, T, S, K_UT>(ctx); }

#if LBPF_STEP_Q == 7
using StepL = D3Q7;
#elif LBPF_STEP_Q == 15
using StepL = D3Q15;
#elif LBPF_STEP_Q == 19
using StepL = D3Q19;
#else
#error "LBPF_STEP_Q must be 7, 15 or 19"
#endif

#if LBPF_STEP_STORAGE == 0
#define LBPF_STEP_TYPES float, float
#elif LBPF_STEP_STORAGE == 1
#define LBPF_STEP_TYPES float, __half
#elif LBPF_STEP_STORAGE == 2
#define LBPF_STEP_TYPES float, __hip_bfloat16
#elif LBPF_STEP_STORAGE == 3
#define LBPF_STEP_TYPES double, double
#else
#error "LBPF_STEP_STORAGE must be an lbpf_storage value"
#endif
template lbpf_status launch_step_s<StepL, LBPF_STEP_TYPES>(lbpf_ctx*);
template lbpf_status launch_phi_s<StepL, LBPF_STEP_TYPES>(lbpf_ctx*);
template lbpf_status launch_ut_s<StepL, LBPF_STEP_TYPES>(lbpf_ctx*);
template hipError_t batch_launch_s<StepL, LBPF_STEP_TYPES>(int, int, const void*, const int2*, int, int,
                                                            hipStream_t);

}  // namespace lbpf_rt
