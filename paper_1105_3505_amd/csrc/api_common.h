// Internal helpers shared by the host-side translation units of the C ABI.
#pragma once

#include <string>

#include "host_math.h"
#include "lfmm.h"

namespace lfmm {

// Largest skeleton size the kernels store per box (expansion vectors hold kMaxRank slots
// at most; the per-plan padded rank is a multiple of 16 up to this).
constexpr int kMaxRank = 64;

// Largest leaf side with a dense-model outgoing operator (Remark 8.2).  Its table holds
// rank x side^2 doubles (48 x 16384 x 8 B = 6.3 MB at side 128).
constexpr int64_t kDenseLeafMax = 128;

extern thread_local std::string g_last_error;
lfmm_status fail(lfmm_status s, const std::string& msg);
lfmm_status validate_options(const lfmm_options* o);
OperatorParams operator_params(const lfmm_options& o);

// Frees a plan whose device work is known to be complete (its last execute's completion
// was observed), without the device-wide synchronisation of lfmm_plan_destroy.
void plan_destroy_completed(lfmm_plan* plan);
// Root-box bits D (smallest with 2^D >= coordinate extent; 32 when the extent exceeds 2^31)
// of K point sets in device memory (n and xy host arrays), computed on the device; waits
// for the stream.
lfmm_status root_bits_of(lfmm_ctx* ctx, int32_t K, const int64_t* n, const int32_t* const* xy, void* stream,
                         int32_t* bits);
// Device of a context.
int ctx_device(const lfmm_ctx* ctx);
// Option flags of a context (LFMM_FLAG_*).
int32_t ctx_flags(const lfmm_ctx* ctx);
// Servers of a context, destroyed with it if still alive.
void ctx_add_server(lfmm_ctx* ctx, lfmm_server* srv);
void ctx_remove_server(lfmm_ctx* ctx, lfmm_server* srv);

}  // namespace lfmm
