// Device-side fill of the synthetic density-fitting factor B[P][mu][nu].
//
// Evaluates exactly the counter-based stream defined in synth/__init__.py
// (SplitMix64 draws, Irwin-Hall(12) normal deviates from 16-bit pieces, the
// host-provided decay/scale table, direct float64 -> bfloat16 round-to-nearest-even),
// so every element equals the host generator's bit for bit.  It exists only so
// that multi-GB inputs need not cross PCIe; it holds none of the PNOF arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double ih12(uint64_t key, uint64_t idx) {
  int64_t s = 0;
  const uint64_t base = idx * 3ull;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const uint64_t d = mix64(key + (base + (uint64_t)t + 1ull) * 0x9E3779B97F4A7C15ull);
    s += (int64_t)(d & 0xFFFFull) + (int64_t)((d >> 16) & 0xFFFFull) +
         (int64_t)((d >> 32) & 0xFFFFull) + (int64_t)(d >> 48);
  }
  return (double)(s - 393210ll) / 65536.0;
}

// Nearest bfloat16 (ties to even) of a float64, returned as its 16-bit pattern.
__device__ __forceinline__ uint16_t f64_to_bf16(double x) {
  if (x == 0.0) return (uint16_t)((__double_as_longlong(x) >> 48) & 0x8000);
  int e;
  (void)frexp(x, &e);                       // |x| in [2^(e-1), 2^e)
  int qe = (e - 1 > -126 ? e - 1 : -126) - 7;
  // Both products are by powers of two, hence exact; rint rounds half to even.
  double r = rint(x * ldexp(1.0, -qe)) * ldexp(1.0, qe);
  float f = (float)r;                       // exact: r is a bfloat16 value
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__global__ void fill_b_kernel(void* __restrict__ out, int out_bf16, const double* __restrict__ fac,
                              uint64_t key, int64_t nbf, int64_t p0, int64_t np_, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t % nbf;
    const int64_t i = (t / nbf) % nbf;
    const int64_t P = p0 + t / (nbf * nbf);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const uint64_t idx = (uint64_t)((P * nbf + lo) * nbf + hi);
    const double v = fac[hi - lo] * ih12(key, idx);
    if (out_bf16)
      reinterpret_cast<uint16_t*>(out)[t] = f64_to_bf16(v);
    else
      reinterpret_cast<double*>(out)[t] = v;
  }
}

}  // namespace

extern "C" {

// Fill rows P in [p0, p0+np) of B into `out` (device, np*nbf*nbf elements, row-major
// [P][mu][nu]); `fac` is the device copy of the nbf-entry factor table; out_bf16 selects
// bfloat16 (1) or float64 (0) storage.  Returns 0 on success, a hipError_t otherwise.
int synth_fill_b(void* out, int out_bf16, const double* fac, uint64_t key, int64_t nbf,
                 int64_t p0, int64_t np_, void* stream) {
  if (!out || !fac || nbf <= 0 || np_ < 0 || p0 < 0) return (int)hipErrorInvalidValue;
  const int64_t total = np_ * nbf * nbf;
  if (total == 0) return 0;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536 * 8) blocks = 65536 * 8;
  hipLaunchKernelGGL(fill_b_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, out,
                     out_bf16, fac, key, nbf, p0, np_, total);
  return (int)hipGetLastError();
}

}  // extern "C"
