// bk_internal.hpp - declarations shared between the translation units of libbesselk.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

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

const RuleTable& rule_table();
const RuleTable* rule_table_dev();
const TemmeCoef& temme_coef();
const TemmeCoef* temme_coef_dev();
void resolve_thresholds(int mode, double L_in, double Lq_in, double* L, double* Lq);

// Records the caller's kernel_events[k] on stream when both events are set
// (hipSuccess otherwise).
inline hipError_t mark_kernel_event(const bk_params* p, int k, hipStream_t stream)
{
    if (!p->kernel_events[0] || !p->kernel_events[1]) return hipSuccess;
    return hipEventRecord((hipEvent_t)p->kernel_events[k], stream);
}

int bk_besselk_learned(const double* nu, const double* x, double* out, int64_t n, const bk_params* prm,
                       double L, double Lq, hipStream_t stream);
int bk_matern_learned(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                      void* out, double L, double Lq, hipStream_t stream);

}  // namespace bk
