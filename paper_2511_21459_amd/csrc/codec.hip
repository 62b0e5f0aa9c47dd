// The 16-bit storage conversions exposed for checking: the device codecs the fusion kernels apply
// when they store and load a value, and their host counterparts (used for the host store and for
// blocks loaded from outside).
#include "mrh_store.h"

namespace mrh {

__global__ __launch_bounds__(256) void k_codec(int32_t storage, int32_t decode, const void* __restrict__ in, void* out,
                                               int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (decode) {
            const uint16_t b = static_cast<const uint16_t*>(in)[i];
            static_cast<float*>(out)[i] = storage == MRH_STORE_F16 ? f16_to_f32(b) : bf16_to_f32(b);
        } else {
            const float x = static_cast<const float*>(in)[i];
            static_cast<uint16_t*>(out)[i] = storage == MRH_STORE_F16 ? f32_to_f16(x) : f32_to_bf16(x);
        }
    }
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_codec_device(int32_t storage, int32_t decode, const void* in_dev, void* out_dev, int64_t n) {
    if ((storage != MRH_STORE_F16 && storage != MRH_STORE_BF16) || n < 0 || (n > 0 && (!in_dev || !out_dev)))
        return MRH_ERR_INVALID_ARG;
    if (n == 0) return MRH_OK;
    const int64_t want = (n + 255) / 256;
    const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(k_codec, dim3(grid), dim3(256), 0, nullptr, storage, decode, in_dev, out_dev, n);
    if (hipGetLastError() != hipSuccess) return MRH_ERR_HIP;
    return hipStreamSynchronize(nullptr) == hipSuccess ? MRH_OK : MRH_ERR_HIP;
}

extern "C" mrh_status mrh_codec_host(int32_t storage, int32_t decode, const void* in, void* out, int64_t n) {
    if ((storage != MRH_STORE_F16 && storage != MRH_STORE_BF16) || n < 0 || (n > 0 && (!in || !out)))
        return MRH_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i) {
        if (decode) {
            const uint16_t b = static_cast<const uint16_t*>(in)[i];
            static_cast<float*>(out)[i] = storage == MRH_STORE_F16 ? h_f16(b) : h_bf16(b);
        } else {
            const float x = static_cast<const float*>(in)[i];
            static_cast<uint16_t*>(out)[i] = storage == MRH_STORE_F16 ? h_to_f16(x) : h_to_bf16(x);
        }
    }
    return MRH_OK;
}
