// bk_internal.hpp - declarations shared between the translation units of libbesselk.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>

#include "../../include/besselk.h"
#include "bk_math.hpp"

namespace bk {

// Default thresholds. Plain: L = 36 ~ -ln(2^-52) (Sec. IV-B takes the window at
// machine epsilon), node target e^-35. Mixed and learned: L = 15, node target
// e^-14.5; the quadrature error is then ~2.5e-7 at most over nu in [0.01, 10],
// x in [1e-4, 1e3], leaving the rest of a 2e-6 relative budget to the FP32
// rounding of the node terms.
constexpr double kDefaultLPlain = 36.0;
constexpr double kDefaultLqPlain = 35.0;
constexpr double kDefaultLMixed = 15.0;
constexpr double kDefaultLqMixed = 14.5;

// The paper's refined algorithm: b = 40 bins on [0, 9] for x >= 0.1, Temme's
// series below (Sec. IV-C, Alg. 2).
constexpr int kPaperBins = 40;
constexpr double kPaperT = 9.0;
constexpr double kPaperTemmeX = 0.1;

void resolve_thresholds(int mode, double L_in, double Lq_in, double* L, double* Lq);

// Records the caller's kernel_events[k] on stream when both events are set
// (hipSuccess otherwise).
inline hipError_t mark_kernel_event(const bk_params* p, int k, hipStream_t stream)
{
    if (!p->kernel_events[0] || !p->kernel_events[1]) return hipSuccess;
    return hipEventRecord((hipEvent_t)p->kernel_events[k], stream);
}

template <typename... P, size_t... I>
inline int launch_args(void (*k)(P...), dim3 grid, dim3 block, hipStream_t stream, std::tuple<P...>& args,
                       std::index_sequence<I...>)
{
    void* ptrs[] = {static_cast<void*>(&std::get<I>(args))...};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, ptrs, 0, stream) == hipSuccess ? BK_OK
                                                                                                       : BK_EHIP;
}

// Enqueues kernel k on stream, its arguments converted to the kernel's parameter
// types. The status is the launch's own (BK_OK or BK_EHIP): no error state left by
// other code is read or cleared.
template <typename... P, typename... A>
inline int launch(void (*k)(P...), dim3 grid, dim3 block, hipStream_t stream, A&&... a)
{
    static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
    std::tuple<P...> args(std::forward<A>(a)...);
    return launch_args(k, grid, block, stream, args, std::index_sequence_for<P...>{});
}

int bk_besselk_learned(const double* nu, const double* x, double* out, int64_t n, const bk_params* prm,
                       double L, double Lq, hipStream_t stream);
// Workspace bytes of the learned Matern form for one call (window table, interval
// plans, wave bitmap); 0 if the sizes are invalid.
size_t matern_learned_workspace_bytes(int64_t n, int32_t tile_size, int32_t lower_only);
int bk_matern_learned(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                      void* out, double L, double Lq, void* workspace, size_t workspace_bytes, hipStream_t stream);
// bk_matern_tiles with the learned form's workspace given explicitly (the caller's,
// or the no-allocation entry point's static scratch).
int matern_tiles_dispatch(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                          void* out, void* workspace, size_t workspace_bytes, hipStream_t stream);

}  // namespace bk
