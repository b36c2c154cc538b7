// Internal declarations of the surrogate kernels (sur_kernels.hip) used by the
// C ABI in sur_api.hip.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sur {

typedef __bf16 bf16;

hipError_t conv(const bf16* in, int cin, const bf16* w, const float* bias, const void* res, const bf16* mask,
                void* out, int out_f32, int relu_in, int dil, int N, int H, int W, hipStream_t s);
hipError_t adjoint_weights(const bf16* w, int cin, bf16* wt, hipStream_t s);
hipError_t wgrad(const bf16* dy, const bf16* in, int cin, int relu_in, int dil, int N, int H, int W, float* part,
                 int groups, float* out, hipStream_t s);
hipError_t bgrad(const bf16* dy, long long npix, float* part, int groups, float* out, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m1, float* m2, bf16* pb, long long n, float lr, float b1, float b2,
                float eps, int t, hipStream_t s);
// The five FP32 state fields of a frame: phi, ux, uy, T, p.
struct State5 {
    const float* v[5];
};
// Scalings of a frame (mirrors sur_scales of the C ABI).
struct Scales {
    float u, dT, t_a, t_b, P, c4, c5;
    float inc[5];
};

hipError_t mse(const float* delta, const float* target, long long npix, int nout, float scale, bf16* grad,
               float* part, int groups, hipStream_t s);
hipError_t pack(const State5& f, long long npix, int w, const Scales& sc, bf16* x, hipStream_t s);
hipError_t pack_target(const State5& f0, const State5& f1, long long npix, const Scales& sc, float* t, hipStream_t s);
hipError_t advance(const float* delta, long long npix, const Scales& sc, const State5& f, hipStream_t s);
hipError_t conv_advance(const bf16* in, const bf16* w, const float* bias, int relu_in, int dil, int H, int W,
                        const Scales& sc, const State5& f, hipStream_t s);
constexpr int kVolPartsApi = 512;  // partials of conv_advance_volume (the column kernel's kVolParts)
// conv_advance (dilation <= 16) that also sums the light-phase volume of the
// updated phi into *vout; vpart holds kVolParts partials and a zero counter.
hipError_t conv_advance_volume(const bf16* in, const bf16* w, const float* bias, int relu_in, int dil, int H, int W,
                               const Scales& sc, const State5& f, double* vpart, double* vout, hipStream_t s);
hipError_t frame_sums(const State5& a, const State5* b, long long npix, int w, const Scales& sc, double* part,
                      int groups, double* out, hipStream_t s);

// Largest partial-sum count of the allocation-free judge, and the devices it
// keeps an address for.
constexpr int kJudgeMaxGroups = 1024;
constexpr int kMaxDevices = 64;
// Device address of the current device's judge scratch (kJudgeMaxGroups * 8
// doubles), looked up on the first call on each device.
hipError_t judge_scratch_ptr(double** out);

}  // namespace sur
