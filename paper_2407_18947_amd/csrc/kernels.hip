// Generic kernels: batched complex GEMM on the matrix cores (FP64 or FP32
// MFMA, complex product as four real products), strided axpy/permute, fill.
#include <algorithm>

#include "common.h"

namespace rtcc3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BK = 16, NT = 256;

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

// Split k = q*K0 + r for 0 <= k < 2^22 without an integer divide: the float
// estimate of the quotient is off by at most one, corrected either way.
__device__ __forceinline__ void split_k(int k, int K0, float inv, int& q, int& r) {
  q = (int)((float)k * inv);
  r = k - q * K0;
  q = r < 0 ? q - 1 : q;
  r = r < 0 ? r + K0 : r;
  q = r >= K0 ? q + 1 : q;
  r = r >= K0 ? r - K0 : r;
}

// One workgroup computes a 64 x BN tile of C for one batch entry.  BN = 64:
// waves arranged 2x2, each owning a 32x32 sub-tile = 2x2 MFMA 16x16 blocks;
// BN = 16 (narrow N, e.g. one occupied index): waves stacked 4x1, each owning
// one 16x16 block.  Every block has a real and an imaginary accumulator:
//   Cre += Are*Bre - Aim*Bim,  Cim += Are*Bim + Aim*Bre.
// MFMA 16x16x4 operand layout: lane l holds A[l%16][l/16] and B[l/16][l%16].
// Result layout: FP32 holds D[4*(l/16)+r][l%16] in register r, FP64 holds
// D[4*r+l/16][l%16] (Frag<T>::row).
//
// Tiles of A and B go through two LDS buffers: while the MFMAs consume one,
// the next tile is loaded into registers and then stored into the other, so
// each K step needs one barrier.  Loads carry no branches: an element outside
// the operand reads the entry's first element and is replaced by zero.
// KFA: A is read with k as the fast thread index (unit stride in k), else m;
// NFB: B is read with n as the fast thread index, else k.
// SEG: the operands come from the K segments of the descriptor (A read with
// k fast, B with n fast).
template <typename T, bool ATOMIC, bool KFA, bool NFB, int BN, bool SEG>
__global__ __launch_bounds__(NT) void zgemm_kernel(GemmDesc d, int ksplit, int kchunk) {
  typedef typename Frag<T>::acc acc_t;
  constexpr int WM = BN == 64 ? 32 : 16, WN = BN == 64 ? 32 : 16;  // wave sub-tile
  constexpr int IB = WM / 16, JB = WN / 16;                         // MFMA blocks per wave
  constexpr int NEB = BN * BK / NT;                                 // B elements per thread
  __shared__ T sA[2][2][BK][BM + 1];  // [buffer][re, im][k][m]
  __shared__ T sB[2][2][BK][BN + 1];  // [buffer][re, im][k][n]

  const int tilesN = (d.N + BN - 1) / BN;
  const int kz = blockIdx.x % ksplit;
  const int tile = blockIdx.x / ksplit;
  const int tm = tile / tilesN, tn = tile % tilesN;
  const int64_t b = (int64_t)blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (b >= d.batch) return;
  const int kbeg = kz * kchunk;
  const int kend = min(d.K, kbeg + kchunk);
  if (kbeg >= kend) return;
  const cplx* A = nullptr;
  const cplx* B = nullptr;
  cplx* C;
  const cplx* Ap[4] = {nullptr, nullptr, nullptr, nullptr};  // K-segment bases of this entry
  const cplx* Bp[4] = {nullptr, nullptr, nullptr, nullptr};
  if (d.bl) {
    const int I = d.bl[4 * b], J = d.bl[4 * b + 1], K = d.bl[4 * b + 2], n = d.bl[4 * b + 3];
    C = d.C + d.cC[0] * I + d.cC[1] * J + d.cC[2] * K + d.cC[3] * n;
    if (SEG) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const GemmDesc::Seg& g = d.seg[s < d.nseg ? s : 0];
        Ap[s] = g.A + g.cA[0] * I + g.cA[1] * J + g.cA[2] * K + g.cA[3] * n;
        Bp[s] = g.B + g.cB[0] * I + g.cB[1] * J + g.cB[2] * K + g.cB[3] * n;
      }
    } else {
      A = d.A + d.cA[0] * I + d.cA[1] * J + d.cA[2] * K + d.cA[3] * n;
      B = d.B + d.cB[0] * I + d.cB[1] * J + d.cB[2] * K + d.cB[3] * n;
    }
  } else {
    A = d.A + b * d.sAb;
    B = d.B + b * d.sBb;
    C = d.C + b * d.sCb;
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / (BN / WN)) * WM, wn = (wave % (BN / WN)) * WN;
  const float invK0 = 1.0f / (float)d.K0;

  // Loader geometry: element r of a thread sits at (akk[r], amm[r]) of the A
  // tile; with KFA all four share one k (one k slot), else one m.
  constexpr int NKA = KFA ? 1 : 4, NMA = KFA ? 4 : 1;
  constexpr int NKB = NFB ? NEB : 1, NNB = NFB ? 1 : NEB;
  int akk[4], amm[4], bkk[NEB], bnn[NEB];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = tid + NT * r;
    amm[r] = KFA ? e / BK : e % BM;
    akk[r] = KFA ? e % BK : e / BM;
  }
#pragma unroll
  for (int r = 0; r < NEB; ++r) {
    const int e = tid + NT * r;
    bnn[r] = NFB ? e % BN : e / BK;
    bkk[r] = NFB ? e / BN : e % BK;
  }
  int64_t aoff[NMA], boff[NNB];
  bool aval[NMA], bval[NNB];
#pragma unroll
  for (int r = 0; r < NMA; ++r) {
    const int m = tm * BM + amm[r];
    aval[r] = m < d.M;
    aoff[r] = aval[r] ? (int64_t)(m / d.M0) * d.sAm1 + (int64_t)(m % d.M0) * d.sAm0 : 0;
  }
#pragma unroll
  for (int r = 0; r < NNB; ++r) {
    const int n = tn * BN + bnn[r];
    bval[r] = n < d.N;
    boff[r] = bval[r] ? (int64_t)(n / d.N0) * d.sBn1 + (int64_t)(n % d.N0) * d.sBn0 : 0;
  }
  // Every load is issued: an element outside the operand reads offset 0 of
  // its entry (the empty asm keeps the compiler from turning the address
  // select back into a branch around the load) and is then replaced by zero.
  cplx av[4], bv[NEB];
  auto fetch = [](const cplx* p, bool ok, int64_t off) {
    int64_t o = ok ? off : 0;
    asm volatile("" : "+v"(o));
    const cplx x = p[o];
    return cplx{ok ? x.re : 0.0, ok ? x.im : 0.0};
  };
  // Segment of k (SEG): unused segments start at INT_MAX.
  const int sk1 = d.nseg > 1 ? d.seg[1].k0 : 0x7fffffff;
  const int sk2 = d.nseg > 2 ? d.seg[2].k0 : 0x7fffffff;
  const int sk3 = d.nseg > 3 ? d.seg[3].k0 : 0x7fffffff;
  auto segof = [&](int k) { return (int)(k >= sk1) + (int)(k >= sk2) + (int)(k >= sk3); };
  auto pick = [](int s, auto x0, auto x1, auto x2, auto x3) { return s == 0 ? x0 : s == 1 ? x1 : s == 2 ? x2 : x3; };
  auto load = [&](int k0) {
    if (SEG) {
      // A: one k per thread (k fast), four rows; B: one column, four k
      const int k = k0 + akk[0];
      const int s = segof(k);
      const int r = k - pick(s, 0, sk1, sk2, sk3);
      const cplx* p = pick(s, Ap[0], Ap[1], Ap[2], Ap[3]);
      const int64_t sm = pick(s, d.seg[0].sAm, d.seg[1].sAm, d.seg[2].sAm, d.seg[3].sAm);
      const int64_t kof = (int64_t)r * pick(s, d.seg[0].sAk, d.seg[1].sAk, d.seg[2].sAk, d.seg[3].sAk);
#pragma unroll
      for (int t = 0; t < 4; ++t) av[t] = fetch(p, k < kend && aval[t], (int64_t)(tm * BM + amm[t]) * sm + kof);
      const int64_t ncol = tn * BN + bnn[0];
#pragma unroll
      for (int t = 0; t < NEB; ++t) {
        const int kb = k0 + bkk[t];
        const int sb = segof(kb);
        const int rb = kb - pick(sb, 0, sk1, sk2, sk3);
        const cplx* pb = pick(sb, Bp[0], Bp[1], Bp[2], Bp[3]);
        const int64_t off = (int64_t)rb * pick(sb, d.seg[0].sBk, d.seg[1].sBk, d.seg[2].sBk, d.seg[3].sBk) +
                            ncol * pick(sb, d.seg[0].sBn, d.seg[1].sBn, d.seg[2].sBn, d.seg[3].sBn);
        bv[t] = fetch(pb, kb < kend && bval[0], off);
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < NKA; ++s) {
      const int k = k0 + akk[s];
      int q, r;
      split_k(k, d.K0, invK0, q, r);
      const int64_t ko = (int64_t)q * d.sAk1 + (int64_t)r * d.sAk0;
#pragma unroll
      for (int t = 0; t < NMA; ++t) {
        const int e = KFA ? t : s;
        av[e] = fetch(A, k < kend && aval[KFA ? t : 0], aoff[KFA ? t : 0] + ko);
      }
    }
#pragma unroll
    for (int s = 0; s < NKB; ++s) {
      const int k = k0 + bkk[s];
      int q, r;
      split_k(k, d.K0, invK0, q, r);
      const int64_t ko = (int64_t)q * d.sBk1 + (int64_t)r * d.sBk0;
#pragma unroll
      for (int t = 0; t < NNB; ++t) {
        const int e = NFB ? s : t;
        bv[e] = fetch(B, k < kend && bval[NFB ? 0 : t], boff[NFB ? 0 : t] + ko);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sA[buf][0][akk[r]][amm[r]] = (T)av[r].re;
      sA[buf][1][akk[r]][amm[r]] = (T)av[r].im;
    }
#pragma unroll
    for (int r = 0; r < NEB; ++r) {
      sB[buf][0][bkk[r]][bnn[r]] = (T)bv[r].re;
      sB[buf][1][bkk[r]][bnn[r]] = (T)bv[r].im;
    }
  };

  acc_t cre[IB][JB], cim[IB][JB];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      cre[i][j] = acc_t{0, 0, 0, 0};
      cim[i][j] = acc_t{0, 0, 0, 0};
    }

  const int nsteps = (kend - kbeg + BK - 1) / BK;
  load(kbeg);
  stash(0);
  __syncthreads();
  // The last step also loads and stores a (fully masked) next tile: the loop
  // body then has no branch, and the buffer it overwrites is no longer read.
  for (int it = 0; it < nsteps; ++it) {
    const int cur = it & 1;
    load(kbeg + (it + 1) * BK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      T ar[IB], ai[IB], nai[IB], br[JB], bi[JB];
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        ar[i] = sA[cur][0][kr][wm + 16 * i + c16];
        ai[i] = sA[cur][1][kr][wm + 16 * i + c16];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        br[j] = sB[cur][0][kr][wn + 16 * j + c16];
        bi[j] = sB[cur][1][kr][wn + 16 * j + c16];
      }
      // four independent MFMAs between two that update the same accumulator
#pragma unroll
      for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) cre[i][j] = Frag<T>::mfma(ar[i], br[j], cre[i][j]);
#pragma unroll
      for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) cim[i][j] = Frag<T>::mfma(ar[i], bi[j], cim[i][j]);
#pragma unroll
      for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) cre[i][j] = Frag<T>::mfma(nai[i], bi[j], cre[i][j]);
#pragma unroll
      for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) cim[i][j] = Frag<T>::mfma(ai[i], br[j], cim[i][j]);
    }
    stash(cur ^ 1);
    __syncthreads();
  }

  const double alr = d.alpha.re, ali = d.alpha.im;
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j)
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

template <typename T, bool ATOMIC, int BN>
void launch_zgemm_l(const GemmDesc& d, dim3 grid, hipStream_t s, int ksplit, int kchunk, bool kfa, bool nfb) {
  if (kfa && nfb)
    hipLaunchKernelGGL((zgemm_kernel<T, ATOMIC, true, true, BN, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  else if (kfa)
    hipLaunchKernelGGL((zgemm_kernel<T, ATOMIC, true, false, BN, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  else if (nfb)
    hipLaunchKernelGGL((zgemm_kernel<T, ATOMIC, false, true, BN, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  else
    hipLaunchKernelGGL((zgemm_kernel<T, ATOMIC, false, false, BN, false>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
}

template <typename T, bool ATOMIC>
void launch_zgemm_t(const GemmDesc& d, dim3 grid, hipStream_t s, int ksplit, int kchunk, bool kfa, bool nfb,
                    int bn) {
  if (d.nseg > 0)
    hipLaunchKernelGGL((zgemm_kernel<T, ATOMIC, true, true, 64, true>), grid, dim3(NT), 0, s, d, ksplit, kchunk);
  else if (bn == 16)
    launch_zgemm_l<T, ATOMIC, 16>(d, grid, s, ksplit, kchunk, kfa, nfb);
  else
    launch_zgemm_l<T, ATOMIC, 64>(d, grid, s, ksplit, kchunk, kfa, nfb);
}

void launch_zgemm(const GemmDesc& d, dim3 grid, hipStream_t s, int ksplit, int kchunk, bool f32, bool atomic,
                  bool kfa, bool nfb, int bn) {
  if (f32) {
    if (atomic)
      launch_zgemm_t<float, true>(d, grid, s, ksplit, kchunk, kfa, nfb, bn);
    else
      launch_zgemm_t<float, false>(d, grid, s, ksplit, kchunk, kfa, nfb, bn);
  } else {
    if (atomic)
      launch_zgemm_t<double, true>(d, grid, s, ksplit, kchunk, kfa, nfb, bn);
    else
      launch_zgemm_t<double, false>(d, grid, s, ksplit, kchunk, kfa, nfb, bn);
  }
}

// The same product with the roles of A and B exchanged: C^T = B^T A^T.
GemmDesc transposed(const GemmDesc& d) {
  GemmDesc t = d;
  t.M = d.N;
  t.N = d.M;
  t.M0 = d.N0;
  t.N0 = d.M0;
  t.A = d.B;
  t.sAm1 = d.sBn1;
  t.sAm0 = d.sBn0;
  t.sAk1 = d.sBk1;
  t.sAk0 = d.sBk0;
  t.sAb = d.sBb;
  t.B = d.A;
  t.sBk1 = d.sAk1;
  t.sBk0 = d.sAk0;
  t.sBn1 = d.sAm1;
  t.sBn0 = d.sAm0;
  t.sBb = d.sAb;
  t.sCm1 = d.sCn1;
  t.sCm0 = d.sCn0;
  t.sCn1 = d.sCm1;
  t.sCn0 = d.sCm0;
  std::copy(d.cB, d.cB + 4, t.cA);
  std::copy(d.cA, d.cA + 4, t.cB);
  return t;
}

}  // namespace

void gemm(const GemmDesc& d0, hipStream_t s) {
  if (d0.M <= 0 || d0.N <= 0 || d0.batch <= 0) return;
  if (d0.K <= 0) return;
  RTCC3_CHECK(d0.M0 >= 1 && d0.N0 >= 1 && d0.K0 >= 1, "gemm: inner extents must be >= 1");
  if (d0.nseg > 0) {
    RTCC3_CHECK(d0.nseg <= 4 && d0.bl && d0.seg[0].k0 == 0 && d0.M0 == d0.M && d0.N0 == d0.N,
                "gemm: bad K segments");
    for (int s = 0; s < d0.nseg; ++s) {
      const int end = s + 1 < d0.nseg ? d0.seg[s + 1].k0 : d0.K;
      RTCC3_CHECK(d0.seg[s].A && d0.seg[s].B && end > d0.seg[s].k0, "gemm: bad K segments");
    }
  }
  RTCC3_CHECK(d0.K < (1 << 22), "gemm: K too long");
  RTCC3_CHECK(!d0.store || !d0.atomic, "gemm: store mode cannot be atomic");
  // A narrow side (at most 16, e.g. one occupied index) goes on N with 64x16
  // tiles; a narrow M is moved there by transposing the product.
  const bool tr = d0.M <= 16 && d0.N > 16 && d0.nseg == 0;
  const GemmDesc d = tr ? transposed(d0) : d0;
  const int bn = d.N <= 16 && d.nseg == 0 ? 16 : 64;  // the segmented kernel has 64-wide tiles
  const int64_t tiles = (int64_t)((d.M + BM - 1) / BM) * ((d.N + bn - 1) / bn);
  // Split K across workgroups when the grid is too small to fill the chip and
  // K is long; the partial products are then added with atomics.
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
  const bool kfa = d.sAk0 == 1, nfb = d.sBn0 == 1;
  launch_zgemm(d, grid, s, ksplit, kchunk, d.prec != 0, atomic, kfa, nfb, bn);
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
