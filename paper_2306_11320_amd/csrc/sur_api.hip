// C ABI of the surrogate kernels (include/surrogate.h): argument checks and
// launches.
#include "surrogate.h"
#include "sur_internal.hpp"

static_assert(SUR_JUDGE_MAX_GROUPS == sur::kJudgeMaxGroups, "judge scratch size");
static_assert(SUR_VOLUME_PARTS == sur::kVolPartsApi, "volume partials");

#include <cstdio>
#include <string>

namespace {
thread_local std::string g_err;

int check(hipError_t e, const char* what)
{
    if (e == hipSuccess) return 0;
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return -3;
}
int bad(const char* what)
{
    g_err = what;
    return -1;
}
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
}  // namespace

using sur::bf16;

extern "C" {

int sur_conv3x3(const void* d_in, int cin, const void* d_w, const float* d_bias, const void* d_res,
                const void* d_mask, void* d_out, int out_f32, int relu_in, int dil, int n, int h, int w, void* stream)
{
    if (!d_in || !d_w || !d_out) return bad("sur_conv3x3: NULL tensor");
    if (cin != 8 && cin != 32) return bad("sur_conv3x3: cin must be 8 or 32");
    if (n < 1 || h < 1 || w < 1) return bad("sur_conv3x3: need n, h, w >= 1");
    if (dil < 1 || dil > w) return bad("sur_conv3x3: need 1 <= dil <= w");
    // 32-pixel segments are numbered with 32-bit integers in the kernel
    if ((long long)n * h * ((w + 31) / 32) >= (1LL << 30)) return bad("sur_conv3x3: more than 2^30 segments");
    if (!aligned16(d_in) || !aligned16(d_w) || !aligned16(d_out) || (d_res && !aligned16(d_res)))
        return bad("sur_conv3x3: in, w, res and out must be 16-byte aligned");
    return check(sur::conv(static_cast<const bf16*>(d_in), cin, static_cast<const bf16*>(d_w), d_bias, d_res,
                           static_cast<const bf16*>(d_mask), d_out, out_f32, relu_in, dil, n, h, w,
                           static_cast<hipStream_t>(stream)),
                 "sur_conv3x3");
}

int sur_adjoint_weights(const void* d_w, int cin, void* d_wt, void* stream)
{
    if (!d_w || !d_wt) return bad("sur_adjoint_weights: NULL tensor");
    if (cin != 8 && cin != 32) return bad("sur_adjoint_weights: cin must be 8 or 32");
    return check(sur::adjoint_weights(static_cast<const bf16*>(d_w), cin, static_cast<bf16*>(d_wt),
                                      static_cast<hipStream_t>(stream)),
                 "sur_adjoint_weights");
}

size_t sur_wgrad_scratch_floats(int cin, int groups) { return (size_t)groups * 32 * 9 * (size_t)cin; }

int sur_weight_grad(const void* d_dy, const void* d_in, int cin, int relu_in, int dil, int n, int h, int w,
                    float* d_part, int groups, float* d_out, void* stream)
{
    if (!d_dy || !d_in || !d_part || !d_out) return bad("sur_weight_grad: NULL tensor");
    if (cin != 8 && cin != 32) return bad("sur_weight_grad: cin must be 8 or 32");
    if (n < 1 || h < 1 || w < 1 || groups < 1) return bad("sur_weight_grad: bad sizes");
    if (dil < 1 || dil > w) return bad("sur_weight_grad: need 1 <= dil <= w");
    return check(sur::wgrad(static_cast<const bf16*>(d_dy), static_cast<const bf16*>(d_in), cin, relu_in, dil, n, h, w,
                            d_part, groups, d_out, static_cast<hipStream_t>(stream)),
                 "sur_weight_grad");
}

int sur_bias_grad(const void* d_dy, int64_t npix, float* d_part, int groups, float* d_out, void* stream)
{
    if (!d_dy || !d_part || !d_out || npix < 1 || groups < 1) return bad("sur_bias_grad: bad arguments");
    return check(sur::bgrad(static_cast<const bf16*>(d_dy), npix, d_part, groups, d_out,
                            static_cast<hipStream_t>(stream)),
                 "sur_bias_grad");
}

int sur_adam(float* d_p, const float* d_g, float* d_m1, float* d_m2, void* d_pb, int64_t n, float lr, float beta1,
             float beta2, float eps, int t, void* stream)
{
    if (!d_p || !d_g || !d_m1 || !d_m2 || !d_pb || n < 1 || t < 1) return bad("sur_adam: bad arguments");
    return check(sur::adam(d_p, d_g, d_m1, d_m2, static_cast<bf16*>(d_pb), n, lr, beta1, beta2, eps, t,
                           static_cast<hipStream_t>(stream)),
                 "sur_adam");
}

int sur_mse(const float* d_delta, const float* d_target, int64_t npix, int nout, float scale, void* d_grad,
            float* d_part, int groups, void* stream)
{
    if (!d_delta || !d_target || !d_grad || !d_part || npix < 1 || groups < 1 || nout < 1 || nout > 32)
        return bad("sur_mse: bad arguments");
    return check(sur::mse(d_delta, d_target, npix, nout, scale, static_cast<bf16*>(d_grad), d_part, groups,
                          static_cast<hipStream_t>(stream)),
                 "sur_mse");
}

namespace {
bool get_state(const float* const* d, sur::State5& out)
{
    if (!d) return false;
    for (int c = 0; c < 5; ++c) {
        out.v[c] = d[c];
        if (!out.v[c]) return false;
    }
    return true;
}
bool get_scales(const sur_scales* s, sur::Scales& out)
{
    if (!s || !(s->u > 0) || !(s->dT > 0) || !(s->P > 0)) return false;
    out = sur::Scales{s->u, s->dT, s->t_a, s->t_b, s->P, s->c4, s->c5, {}};
    for (int c = 0; c < 5; ++c) {
        out.inc[c] = s->inc[c];
        if (!(out.inc[c] > 0)) return false;
    }
    return true;
}
}  // namespace

int sur_pack(const float* const* d_f, int h, int w, const sur_scales* scales, void* d_x, void* stream)
{
    sur::State5 f;
    sur::Scales sc;
    if (!get_state(d_f, f) || !get_scales(scales, sc) || !d_x || h < 1 || w < 1) return bad("sur_pack: bad arguments");
    return check(sur::pack(f, (long long)h * w, w, sc, static_cast<bf16*>(d_x), static_cast<hipStream_t>(stream)),
                 "sur_pack");
}

int sur_pack_target(const float* const* d_f0, const float* const* d_f1, int64_t npix, const sur_scales* scales,
                    float* d_t, void* stream)
{
    sur::State5 f0, f1;
    sur::Scales sc;
    if (!get_state(d_f0, f0) || !get_state(d_f1, f1) || !get_scales(scales, sc) || !d_t || npix < 1)
        return bad("sur_pack_target: bad arguments");
    return check(sur::pack_target(f0, f1, npix, sc, d_t, static_cast<hipStream_t>(stream)), "sur_pack_target");
}

int sur_advance(const float* d_delta, int64_t npix, const sur_scales* scales, float* const* d_f, void* stream)
{
    sur::State5 f;
    sur::Scales sc;
    if (!d_delta || !get_state(d_f, f) || !get_scales(scales, sc) || npix < 1) return bad("sur_advance: bad arguments");
    return check(sur::advance(d_delta, npix, sc, f, static_cast<hipStream_t>(stream)), "sur_advance");
}

int sur_conv3x3_advance(const void* d_in, const void* d_w, const float* d_bias, int relu_in, int dil, int h, int w,
                        const sur_scales* scales, float* const* d_f, void* stream)
{
    sur::State5 f;
    sur::Scales sc;
    if (!d_in || !d_w || !get_state(d_f, f) || !get_scales(scales, sc)) return bad("sur_conv3x3_advance: bad arguments");
    if (h < 1 || w < 1) return bad("sur_conv3x3_advance: need h, w >= 1");
    if (dil < 1 || dil > w) return bad("sur_conv3x3_advance: need 1 <= dil <= w");
    if ((long long)h * ((w + 31) / 32) >= (1LL << 30)) return bad("sur_conv3x3_advance: more than 2^30 segments");
    if (!aligned16(d_in) || !aligned16(d_w)) return bad("sur_conv3x3_advance: in and w must be 16-byte aligned");
    return check(sur::conv_advance(static_cast<const bf16*>(d_in), static_cast<const bf16*>(d_w), d_bias, relu_in, dil,
                                   h, w, sc, f, static_cast<hipStream_t>(stream)),
                 "sur_conv3x3_advance");
}

int sur_conv3x3_advance_volume(const void* d_in, const void* d_w, const float* d_bias, int relu_in, int dil, int h,
                               int w, const sur_scales* scales, float* const* d_f, double* d_part, double* d_vol,
                               void* stream)
{
    sur::State5 f;
    sur::Scales sc;
    if (!d_in || !d_w || !get_state(d_f, f) || !get_scales(scales, sc) || !d_part || !d_vol)
        return bad("sur_conv3x3_advance_volume: bad arguments");
    if (h < 1 || w < 1) return bad("sur_conv3x3_advance_volume: need h, w >= 1");
    if (dil < 1 || dil > w || dil > 16) return bad("sur_conv3x3_advance_volume: need 1 <= dil <= min(w, 16)");
    if ((long long)h * ((w + 31) / 32) >= (1LL << 30)) return bad("sur_conv3x3_advance_volume: more than 2^30 segments");
    if (!aligned16(d_in) || !aligned16(d_w) || (reinterpret_cast<uintptr_t>(d_part) & 7))
        return bad("sur_conv3x3_advance_volume: in and w must be 16-byte aligned, part 8-byte aligned");
    return check(sur::conv_advance_volume(static_cast<const bf16*>(d_in), static_cast<const bf16*>(d_w), d_bias,
                                          relu_in, dil, h, w, sc, f, d_part, d_vol, static_cast<hipStream_t>(stream)),
                 "sur_conv3x3_advance_volume");
}

int sur_light_volume(const float* d_phi, int h, int w, double* d_part, int groups, double* d_out, void* stream)
{
    if (!d_phi || !d_part || !d_out || h < 1 || w < 1 || groups < 1) return bad("sur_light_volume: bad arguments");
    sur::State5 f{{d_phi, d_phi, d_phi, d_phi, d_phi}};
    sur::Scales sc{};
    return check(sur::frame_sums(f, nullptr, (long long)h * w, w, sc, d_part, groups, d_out,
                                 static_cast<hipStream_t>(stream)),
                 "sur_light_volume");
}

int sur_judge(const float* const* d_a, const float* const* d_b, int h, int w, const sur_scales* scales,
              double* d_part, int groups, double* d_out, void* stream)
{
    sur::State5 a, b;
    sur::Scales sc;
    if (!get_state(d_a, a) || !get_state(d_b, b) || !get_scales(scales, sc) || !d_part || !d_out || h < 1 || w < 1 ||
        groups < 1)
        return bad("sur_judge: bad arguments");
    return check(sur::frame_sums(a, &b, (long long)h * w, w, sc, d_part, groups, d_out,
                                 static_cast<hipStream_t>(stream)),
                 "sur_judge");
}

int sur_judge_noscratch(const float* const* d_a, const float* const* d_b, int h, int w, const sur_scales* scales,
                        int groups, double* d_out, void* stream)
{
    sur::State5 a, b;
    sur::Scales sc;
    if (!get_state(d_a, a) || !get_state(d_b, b) || !get_scales(scales, sc) || !d_out || h < 1 || w < 1)
        return bad("sur_judge_noscratch: bad arguments");
    if (groups < 1 || groups > SUR_JUDGE_MAX_GROUPS) {
        char msg[128];
        snprintf(msg, sizeof(msg), "sur_judge_noscratch: groups %d outside [1, %d]", groups, SUR_JUDGE_MAX_GROUPS);
        return bad(msg);
    }
    double* part = nullptr;
    int rc = check(sur::judge_scratch_ptr(&part), "sur_judge_noscratch: address of the static scratch");
    if (rc) return rc;
    return check(sur::frame_sums(a, &b, (long long)h * w, w, sc, part, groups, d_out, static_cast<hipStream_t>(stream)),
                 "sur_judge_noscratch");
}

const char* sur_last_error(void) { return g_err.c_str(); }

}  // extern "C"
