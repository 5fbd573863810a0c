// The complex-GEMM self-test without device allocation: the operands and the
// product are staged in a file-scope device array instead of buffers
// allocated per call.
#include <mutex>
#include <string>

#include "../../include/rtcc3.h"
#include "common.h"

namespace rtcc3 {

namespace {

// Staging area: A, B and C of one call, in complex elements (64 MiB).  Each
// device the library runs on holds its own copy until the process ends.
constexpr int64_t kScratchElems = (int64_t)1 << 22;
static __device__ __align__(256) cplx scratch[kScratchElems];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
cplx* g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's scratch array, looked up once per device
// with that device current.  In host code the array's name is not a device
// address: only this pointer is passed to kernels and copies.
cplx* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    RTCC3_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RTCC3_CHECK(p != nullptr, "zgemm_selftest_noalloc: no device address for the scratch array");
    g_ptr[dev] = (cplx*)p;
  }
  return g_ptr[dev];
}

}  // namespace

}  // namespace rtcc3

using namespace rtcc3;

extern "C" int rtcc3_zgemm_selftest_noalloc(int M, int N, int K, int precision, const rtcc3_c64* A,
                                            const rtcc3_c64* B, rtcc3_c64* Cout) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !Cout) {
    set_thread_error("bad gemm arguments");
    return RTCC3_EINVAL;
  }
  if (precision < RTCC3_FP64 || precision > RTCC3_BF16X2) {
    set_thread_error("unknown precision");
    return RTCC3_EINVAL;
  }
  const int64_t nA = (int64_t)M * K, nB = (int64_t)K * N, nC = (int64_t)M * N;
  if (nA + nB + nC > kScratchElems) {
    set_thread_error("zgemm_selftest_noalloc: M*K + K*N + M*N = " + std::to_string(nA + nB + nC) +
                     " complex elements exceeds the staging area of " + std::to_string(kScratchElems));
    return RTCC3_EINVAL;
  }
  try {
    int dev = 0;
    RTCC3_HIP(hipGetDevice(&dev));
    RTCC3_CHECK(dev >= 0 && dev < kMaxDevices, "zgemm_selftest_noalloc: device index out of range");
    cplx* base = scratch_ptr(dev);
    cplx *dA = base, *dB = base + nA, *dC = base + nA + nB;
    hipStream_t s = nullptr;
    RTCC3_HIP(hipMemcpyAsync(dA, A, sizeof(cplx) * nA, hipMemcpyHostToDevice, s));
    RTCC3_HIP(hipMemcpyAsync(dB, B, sizeof(cplx) * nB, hipMemcpyHostToDevice, s));
    // the array keeps the last call's contents: the product accumulates into C
    fill(dC, nC, cplx{0, 0}, s);
    GemmDesc g = {};
    g.M = M;
    g.N = N;
    g.K = K;
    g.M0 = M;
    g.N0 = N;
    g.K0 = K;
    g.batch = 1;
    g.A = dA;
    g.sAm0 = K;
    g.sAk0 = 1;
    g.B = dB;
    g.sBk0 = N;
    g.sBn0 = 1;
    g.C = dC;
    g.sCm0 = N;
    g.sCn0 = 1;
    g.alpha = cplx{1, 0};
    g.prec = precision;
    g.force_prec = 1;
    gemm(g, s);
    RTCC3_HIP(hipMemcpyAsync(Cout, dC, sizeof(cplx) * nC, hipMemcpyDeviceToHost, s));
    RTCC3_HIP(hipStreamSynchronize(s));
    return RTCC3_OK;
  } catch (const Error& ex) {
    set_thread_error(ex.what());
    return ex.code;
  } catch (const std::exception& ex) {
    set_thread_error(ex.what());
    return RTCC3_EDEVICE;
  }
}
