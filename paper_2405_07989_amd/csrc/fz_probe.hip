// fz_probe.hip -- the device's sustained int32 vector-ALU issue rate, the
// ceiling the count walker is compared with.  Every lane runs eight
// independent chains of v_add_u32 (no dependence between consecutive
// instructions of a wave, no memory traffic in the loop), so the rate is the
// vector units' issue rate for a plain 32-bit integer add.  And the rate at
// which the device writes a large buffer to HBM, the ceiling the store walker
// is compared with: a grid-stride loop of 16-byte stores, nothing read.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fz.h"
#include "fz_host.h"

namespace {

constexpr uint32_t kProbeWg = 256;
constexpr uint32_t kProbeChains = 8;
constexpr uint32_t kProbeUnroll = 32; // adds per chain per loop trip

__global__ void __launch_bounds__(kProbeWg) fz_valu_probe_kernel(uint32_t *out, uint32_t trips,
                                                                uint32_t seed)
{
    uint32_t a[kProbeChains], b[kProbeChains];
#pragma unroll
    for (uint32_t c = 0; c < kProbeChains; ++c) {
        a[c] = threadIdx.x * (c + 1) + seed;
        b[c] = seed ^ (c * 0x9E3779B9u);
    }
    for (uint32_t t = 0; t < trips; ++t) {
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; ++u) {
#pragma unroll
            for (uint32_t c = 0; c < kProbeChains; ++c)
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b[c]));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (uint32_t c = 0; c < kProbeChains; ++c) r ^= a[c];
    if (r == 0x5EED5EEDu) out[0] = r; // keeps the chains live; practically never taken
}

// Every lane writes 16 bytes per store, consecutive lanes consecutive
// addresses (1 KiB per wave instruction), over the whole buffer.
__global__ void __launch_bounds__(kProbeWg) fz_write_probe_kernel(uint4 *buf, uint64_t n16,
                                                                 uint32_t seed)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const uint32_t v = (uint32_t)i ^ seed;
        buf[i] = make_uint4(v, v + 1, v + 2, v + 3);
    }
}

} // namespace

extern "C" int fz_probe_hbm_write(uint64_t bytes, double *bytes_per_s, double *ms)
{
    if (bytes_per_s == nullptr || bytes < (1u << 20)) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(fzh::g_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fzh::dev_err_at(e, "hipGetDevice", __LINE__);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fzh::dev_err_at(e, "hipGetDeviceProperties", __LINE__);
    const uint64_t n16 = bytes / 16;
    const uint32_t blocks = (uint32_t)prop.multiProcessorCount * 32;
    uint4 *buf = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;
    int rc = FZ_OK;
    float best = 0;
    if ((e = hipMalloc(&buf, n16 * 16)) != hipSuccess || (e = hipEventCreate(&a)) != hipSuccess ||
        (e = hipEventCreate(&b)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
        rc = fzh::dev_err_at(e, "probe setup", __LINE__);
    } else {
        for (int rep = 0; rep < 4; ++rep) { // the first is a warm-up
            float t = 0;
            if ((e = hipEventRecord(a, s)) != hipSuccess) break;
            hipLaunchKernelGGL(fz_write_probe_kernel, dim3(blocks), dim3(kProbeWg), 0, s, buf, n16,
                               (uint32_t)rep);
            if ((e = hipGetLastError()) != hipSuccess) break;
            if ((e = hipEventRecord(b, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            if ((e = hipEventElapsedTime(&t, a, b)) != hipSuccess) break;
            if (rep > 0 && (best == 0 || t < best)) best = t;
        }
        if (e != hipSuccess) rc = fzh::dev_err_at(e, "probe launch", __LINE__);
    }
    if (s) (void)hipStreamSynchronize(s);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (buf) (void)hipFree(buf);
    if (rc != FZ_OK) return rc;
    if (best <= 0) return FZ_EINTERNAL;
    *bytes_per_s = (double)(n16 * 16) / (best * 1e-3);
    if (ms) *ms = best;
    return FZ_OK;
}

extern "C" int fz_probe_int_valu(double *lane_ops_per_s, double *ms)
{
    if (lane_ops_per_s == nullptr) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(fzh::g_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fzh::dev_err_at(e, "hipGetDevice", __LINE__);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fzh::dev_err_at(e, "hipGetDeviceProperties", __LINE__);
    // enough workgroups to fill every CU at full occupancy, several times over
    const uint32_t blocks = (uint32_t)prop.multiProcessorCount * 32;
    const uint32_t trips = 4096;
    uint32_t *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;
    int rc = FZ_OK;
    float best = 0;
    if ((e = hipMalloc(&out, sizeof(uint32_t))) != hipSuccess ||
        (e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
        rc = fzh::dev_err_at(e, "probe setup", __LINE__);
    } else {
        for (int rep = 0; rep < 4; ++rep) { // the first is a warm-up
            float t = 0;
            if ((e = hipEventRecord(a, s)) != hipSuccess) break;
            hipLaunchKernelGGL(fz_valu_probe_kernel, dim3(blocks), dim3(kProbeWg), 0, s, out, trips,
                               (uint32_t)rep);
            if ((e = hipGetLastError()) != hipSuccess) break;
            if ((e = hipEventRecord(b, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            if ((e = hipEventElapsedTime(&t, a, b)) != hipSuccess) break;
            if (rep > 0 && (best == 0 || t < best)) best = t;
        }
        if (e != hipSuccess) rc = fzh::dev_err_at(e, "probe launch", __LINE__);
    }
    if (s) (void)hipStreamSynchronize(s);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (rc != FZ_OK) return rc;
    if (best <= 0) return FZ_EINTERNAL;
    const double ops = (double)blocks * kProbeWg * trips * kProbeUnroll * kProbeChains;
    *lane_ops_per_s = ops / (best * 1e-3);
    if (ms) *ms = best;
    return FZ_OK;
}
