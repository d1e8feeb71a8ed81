// bk_internal.hpp - declarations shared between the translation units of libbesselk.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "../../include/besselk.h"
#include "bk_math.hpp"

namespace bk {

// Default thresholds. Plain: L = -ln(2^-52) + 2 (Sec. IV-B takes the window at
// machine epsilon; 2 nats of margin), node target e^-36.5. Mixed and learned:
// L = 16, node target e^-15.4, sized for a 2e-6 relative error budget that also
// holds the FP32 rounding of the node terms.
constexpr double kDefaultLPlain = 38.0;
constexpr double kDefaultLqPlain = 36.5;
constexpr double kDefaultLMixed = 16.0;
constexpr double kDefaultLqMixed = 15.4;

const RuleTable& rule_table();
void resolve_thresholds(int mode, double L_in, double Lq_in, double* L, double* Lq);

int bk_besselk_learned(const double* nu, const double* x, double* out, int64_t n, const bk_params* prm,
                       double L, double Lq, hipStream_t stream);
int bk_matern_learned(const bk_locs* locs, const bk_params* prm, int32_t tile_size, int32_t lower_only,
                      void* out, double L, double Lq, hipStream_t stream);

}  // namespace bk
