// Generic kernels: batched complex GEMM on the matrix cores (FP64 or FP32
// MFMA, complex product as four real products), strided axpy/permute, fill.
#include <algorithm>

#include "common.h"

namespace rtcc3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <typename T>
struct Frag;
template <>
struct Frag<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Frag<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ __forceinline__ void atomic_add_cplx(cplx* p, double re, double im) {
  unsafeAtomicAdd(&p->re, re);
  unsafeAtomicAdd(&p->im, im);
}

// One workgroup computes a 64x64 tile of C for one batch entry.  Waves are
// arranged 2x2, each owning a 32x32 sub-tile = 2x2 MFMA 16x16 blocks with a
// real and an imaginary accumulator:
//   Cre += Are*Bre - Aim*Bim,  Cim += Are*Bim + Aim*Bre.
// MFMA 16x16x4 operand layout: lane l holds A[l%16][l/16] and B[l/16][l%16].
// Result layout: FP32 holds D[4*(l/16)+r][l%16] in register r, FP64 holds
// D[4*r+l/16][l%16] (Frag<T>::row).
template <typename T, bool ATOMIC>
__global__ __launch_bounds__(NT) void zgemm_kernel(GemmDesc d, int ksplit, int kchunk) {
  typedef typename Frag<T>::acc acc_t;
  __shared__ T sAr[BK][BM + 1], sAi[BK][BM + 1], sBr[BK][BN + 1], sBi[BK][BN + 1];

  const int tilesN = (d.N + BN - 1) / BN;
  const int kz = blockIdx.x % ksplit;
  const int tile = blockIdx.x / ksplit;
  const int tm = tile / tilesN, tn = tile % tilesN;
  const int64_t b = (int64_t)blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (b >= d.batch) return;
  const int kbeg = kz * kchunk;
  const int kend = min(d.K, kbeg + kchunk);
  if (kbeg >= kend) return;
  const cplx* __restrict__ A;
  const cplx* __restrict__ B;
  const cplx* __restrict__ A2 = nullptr;
  const cplx* __restrict__ B2 = nullptr;
  cplx* __restrict__ C;
  if (d.bl) {
    const int I = d.bl[4 * b], J = d.bl[4 * b + 1], K = d.bl[4 * b + 2], n = d.bl[4 * b + 3];
    A = d.A + d.cA[0] * I + d.cA[1] * J + d.cA[2] * K + d.cA[3] * n;
    B = d.B + d.cB[0] * I + d.cB[1] * J + d.cB[2] * K + d.cB[3] * n;
    C = d.C + d.cC[0] * I + d.cC[1] * J + d.cC[2] * K + d.cC[3] * n;
    if (d.kseg) {
      A2 = d.A2 + d.cA2[0] * I + d.cA2[1] * J + d.cA2[2] * K + d.cA2[3] * n;
      B2 = d.B2 + d.cB2[0] * I + d.cB2[1] * J + d.cB2[2] * K + d.cB2[3] * n;
    }
  } else {
    A = d.A + b * d.sAb;
    B = d.B + b * d.sBb;
    C = d.C + b * d.sCb;
    if (d.kseg) {
      A2 = d.A2 + b * d.sAb;
      B2 = d.B2 + b * d.sBb;
    }
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  // loader geometry: 4 elements of each tile per thread, the fast thread
  // index along the operand's unit-stride dimension when there is one
  const bool kfastA = (d.sAk0 == 1);
  const bool nfastB = (d.sBn0 == 1);
  int amm[4], akk[4], bnn[4], bkk[4];
  int64_t aoff[4], boff[4];
  bool aval[4], bval[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = tid + NT * r;
    amm[r] = kfastA ? e / BK : e % BM;
    akk[r] = kfastA ? e % BK : e / BM;
    const int m = tm * BM + amm[r];
    aval[r] = m < d.M;
    aoff[r] = aval[r] ? (int64_t)(m / d.M0) * d.sAm1 + (int64_t)(m % d.M0) * d.sAm0 : 0;
    bnn[r] = nfastB ? e % BN : e / BK;
    bkk[r] = nfastB ? e / BN : e % BK;
    const int n = tn * BN + bnn[r];
    bval[r] = n < d.N;
    boff[r] = bval[r] ? (int64_t)(n / d.N0) * d.sBn1 + (int64_t)(n % d.N0) * d.sBn0 : 0;
  }

  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = acc_t{0, 0, 0, 0};
      cim[i][j] = acc_t{0, 0, 0, 0};
    }

  cplx av[4], bv[4];
  const int kseg = d.kseg;
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int ka = k0 + akk[r];
      av[r] = cplx{0.0, 0.0};
      if (aval[r] && ka < kend) {
        const cplx* pa = A;
        if (kseg && ka >= kseg) {
          pa = A2;
          ka -= kseg;
        }
        av[r] = pa[aoff[r] + (int64_t)(ka / d.K0) * d.sAk1 + (int64_t)(ka % d.K0) * d.sAk0];
      }
      int kb = k0 + bkk[r];
      bv[r] = cplx{0.0, 0.0};
      if (bval[r] && kb < kend) {
        const cplx* pb = B;
        if (kseg && kb >= kseg) {
          pb = B2;
          kb -= kseg;
        }
        bv[r] = pb[boff[r] + (int64_t)(kb / d.K0) * d.sBk1 + (int64_t)(kb % d.K0) * d.sBk0];
      }
    }
  };

  load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sAr[akk[r]][amm[r]] = (T)av[r].re;
      sAi[akk[r]][amm[r]] = (T)av[r].im;
      sBr[bkk[r]][bnn[r]] = (T)bv[r].re;
      sBi[bkk[r]][bnn[r]] = (T)bv[r].im;
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);  // next tile in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      T ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = sAr[kr][wm + 16 * i + c16];
        ai[i] = sAi[kr][wm + 16 * i + c16];
        nai[i] = -ai[i];
        br[i] = sBr[kr][wn + 16 * i + c16];
        bi[i] = sBi[kr][wn + 16 * i + c16];
      }
      // four independent MFMAs between two that update the same accumulator
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cre[i][j] = Frag<T>::mfma(ar[i], br[j], cre[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cim[i][j] = Frag<T>::mfma(ar[i], bi[j], cim[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cre[i][j] = Frag<T>::mfma(nai[i], bi[j], cre[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cim[i][j] = Frag<T>::mfma(ai[i], br[j], cim[i][j]);
    }
  }

  const double alr = d.alpha.re, ali = d.alpha.im;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = tm * BM + wm + 16 * i + Frag<T>::row(lane, r);
        const int n = tn * BN + wn + 16 * j + (lane & 15);
        if (m < d.M && n < d.N) {
          const double xr = (double)cre[i][j][r], xi = (double)cim[i][j][r];
          const double vr = alr * xr - ali * xi, vi = alr * xi + ali * xr;
          cplx* p = C + (int64_t)(m / d.M0) * d.sCm1 + (int64_t)(m % d.M0) * d.sCm0 +
                    (int64_t)(n / d.N0) * d.sCn1 + (int64_t)(n % d.N0) * d.sCn0;
          if (ATOMIC) {
            atomic_add_cplx(p, vr, vi);
          } else if (d.store) {
            *p = cplx{vr, vi};
          } else {
            cplx c = *p;
            c.re += vr;
            c.im += vi;
            *p = c;
          }
        }
      }
}

__global__ void axpy_kernel(AxpyDesc d, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e, ox = 0, oy = 0;
    for (int k = d.nd - 1; k >= 0; --k) {
      const int64_t q = r % d.shape[k];
      r /= d.shape[k];
      ox += q * d.sx[k];
      oy += q * d.sy[k];
    }
    const cplx x = d.X[ox];
    cplx y = d.Y[oy];
    y.re += d.alpha.re * x.re - d.alpha.im * x.im;
    y.im += d.alpha.re * x.im + d.alpha.im * x.re;
    d.Y[oy] = y;
  }
}

__global__ void fill_kernel(cplx* p, int64_t n, cplx v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

void gemm(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  if (d.K <= 0) return;
  RTCC3_CHECK(d.M0 >= 1 && d.N0 >= 1 && d.K0 >= 1, "gemm: inner extents must be >= 1");
  const int64_t tiles = (int64_t)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  // Split K across workgroups when the grid is too small to fill the chip and
  // K is long; the partial products are then added with atomics.
  RTCC3_CHECK(!d.kseg || (d.K == 2 * d.kseg && d.A2 && d.B2), "gemm: bad K segments");
  RTCC3_CHECK(!d.store || !d.atomic, "gemm: store mode cannot be atomic");
  int ksplit = 1;
  const int64_t wgs = tiles * d.batch;
  if (!d.store && wgs < 512 && d.K >= 8 * BK) {
    const int64_t want = (1024 + wgs - 1) / wgs;
    const int64_t maxs = d.K / (4 * BK);
    ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(want, maxs));
  }
  const int kchunk = (int)((((int64_t)d.K + ksplit - 1) / ksplit + BK - 1) / BK * BK);
  RTCC3_CHECK(tiles * ksplit < (1LL << 31), "gemm: too many tiles");
  int64_t by = d.batch, bz = 1;
  while (by > 65535) {
    by = (by + 1) / 2;
    bz *= 2;
  }
  dim3 grid((unsigned)(tiles * ksplit), (unsigned)by, (unsigned)bz);
  const bool atomic = d.atomic || ksplit > 1;
  if (d.prec == 0) {
    if (atomic)
      hipLaunchKernelGGL((zgemm_kernel<double, true>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
    else
      hipLaunchKernelGGL((zgemm_kernel<double, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  } else {
    if (atomic)
      hipLaunchKernelGGL((zgemm_kernel<float, true>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
    else
      hipLaunchKernelGGL((zgemm_kernel<float, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  }
  RTCC3_HIP(hipGetLastError());
}

void axpy_strided(const AxpyDesc& d, hipStream_t s) {
  int64_t total = 1;
  for (int k = 0; k < d.nd; ++k) total *= d.shape[k];
  if (total <= 0) return;
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, d, total);
  RTCC3_HIP(hipGetLastError());
}

void fill(cplx* p, int64_t n, cplx val, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, val);
  RTCC3_HIP(hipGetLastError());
}

}  // namespace rtcc3
