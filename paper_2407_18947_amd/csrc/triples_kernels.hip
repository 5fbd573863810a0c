// Element-wise and reduction kernels of the triples engine (one block of
// [v,v,v] per ordered occupied triple n, row-major [a][b][c]).
#include "triples_kernels.h"

namespace rtcc3 {

namespace {

__device__ __forceinline__ cplx cadd(cplx x, cplx y) { return cplx{x.re + y.re, x.im + y.im}; }
__device__ __forceinline__ cplx csub(cplx x, cplx y) { return cplx{x.re - y.re, x.im - y.im}; }
__device__ __forceinline__ cplx cmul(cplx x, cplx y) {
  return cplx{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re};
}
__device__ __forceinline__ cplx cscale(double s, cplx x) { return cplx{s * x.re, s * x.im}; }
__device__ __forceinline__ void catomic(cplx* p, cplx x) {
  unsafeAtomicAdd(&p->re, x.re);
  unsafeAtomicAdd(&p->im, x.im);
}

// Contractions with one free virtual index per block (I,J,K), all from one
// coalesced sweep over t[x][y][z] (z fastest), slab by slab in x:
//   flags&1: X1[I][a]      += sum_bc t[a,b,c] L[J,b,K,c]  - sum_bc t[c,b,a] L[J,b,K,c]
//            X2p[I,J][a,b] += sum_c  t[a,b,c] f~[K,c]     - sum_c  t[c,b,a] f~[K,c]
//   flags&2: Z[I][a]       += sum_bc t[a,b,c] l2[J,K,b,c] - sum_bc t[b,a,c] l2[J,K,b,c]
// In sweep coordinates (x,y,z) the six pieces are: X1a[x] = sum_yz t L[y][z],
// X1b[z] = sum_xy t L[y][x], X2a[x][y] = sum_z t f[z], X2b[z][y] = sum_x t f[x],
// Za[x] = sum_yz t l2[y][z], Zb[y] = sum_xz t l2[x][z].
// Same contractions, one (block, a) per workgroup; used when v*v is too large for
// the slab buffer of small_t3_kernel.
// Contractions with one free virtual index per block (I,J,K):
//   flags&1: X1[I][a]     += sum_bc (t[a,b,c] - t[c,b,a]) L[J,b,K,c]
//            X2p[I,J][a,b]+= sum_c  (t[a,b,c] - t[c,b,a]) f~[K, c]
//   flags&2: Z[I][a]      += sum_bc (t[a,b,c] - t[b,a,c]) l2[J,K,b,c]
__global__ void small_t3_simple_kernel(const cplx* __restrict__ T, const int* __restrict__ bl, const cplx* __restrict__ Lov,
                                const cplx* __restrict__ F, const cplx* __restrict__ l2, cplx* __restrict__ X1,
                                cplx* __restrict__ X2p, cplx* __restrict__ Z, int o, int v, int flags) {
  const int q = blockIdx.y, a = blockIdx.x;
  const int I = bl[4 * q], J = bl[4 * q + 1], K = bl[4 * q + 2], n = bl[4 * q + 3];
  const int64_t v3 = (int64_t)v * v * v;
  const int nn = o + v;
  const cplx* t = T + (int64_t)n * v3;
  cplx x1{0, 0}, z{0, 0};
  for (int b = threadIdx.x; b < v; b += blockDim.x) {
    cplx x2f{0, 0};
    const cplx* Lb = Lov + (((int64_t)J * v + b) * o + K) * v;
    const cplx* l2b = l2 + (((int64_t)J * o + K) * v + b) * v;
    for (int c = 0; c < v; ++c) {
      const cplx tabc = t[((int64_t)a * v + b) * v + c];
      if (flags & 1) {
        const cplx tz = csub(tabc, t[((int64_t)c * v + b) * v + a]);
        x1 = cadd(x1, cmul(tz, Lb[c]));
        x2f = cadd(x2f, cmul(tz, F[(int64_t)K * nn + o + c]));
      }
      if (flags & 2) z = cadd(z, cmul(csub(tabc, t[((int64_t)b * v + a) * v + c]), l2b[c]));
    }
    if (flags & 1) catomic(&X2p[(((int64_t)I * o + J) * v + a) * v + b], x2f);
  }
  __shared__ cplx red[2][256];
  red[0][threadIdx.x] = x1;
  red[1][threadIdx.x] = z;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = cadd(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = cadd(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (flags & 1) catomic(&X1[(int64_t)I * v + a], red[0][0]);
    if (flags & 2) catomic(&Z[(int64_t)I * v + a], red[1][0]);
  }
}

// One workgroup of SW_NW waves per block and chunk of x (blockIdx.y); lane = z
// (unit stride), wave w owns the rows y = w, w+SW_NW, ... (v <= 64).  Sums
// over z are wave reductions, sums over x stay in registers (a chunk's
// partial sums are added atomically), sums over y go through LDS at the end.
constexpr int SW_NW = 8;
constexpr int SW_MAXY = 8;
constexpr int SW_XCHUNK = 16;  // x values per workgroup

__global__ __launch_bounds__(64 * SW_NW) void small_t3_wave_kernel(const cplx* __restrict__ T, const int* __restrict__ bl,
                                                              const cplx* __restrict__ Lov, const cplx* __restrict__ F,
                                                              const cplx* __restrict__ l2, cplx* __restrict__ X1,
                                                              cplx* __restrict__ X2p, cplx* __restrict__ Z, int o,
                                                              int v, int flags) {
  __shared__ cplx sx[2][SW_NW][64];  // per-wave partials of X1a[x], Za[x]
  __shared__ cplx sz[SW_NW][64];     // per-wave partials of X1b[z]
  const int q = blockIdx.x;
  const int xb = blockIdx.y * SW_XCHUNK, xe = min(v, xb + SW_XCHUNK);  // this workgroup's x
  const int I = bl[4 * q], J = bl[4 * q + 1], K = bl[4 * q + 2], n = bl[4 * q + 3];
  const int64_t v2 = (int64_t)v * v, v3 = v2 * v;
  const int nn = o + v;
  const cplx* t = T + (int64_t)n * v3;
  const cplx* fK = F + (int64_t)K * nn + o;
  const cplx* l2JK = l2 + ((int64_t)J * o + K) * v2;
  const cplx* LJ = Lov + (int64_t)J * v * o * v + (int64_t)K * v;  // L[J,y,K,z] = LJ[y*o*v + z]
  const int64_t Ly = (int64_t)o * v;
  const bool doX = flags & 1, doZ = flags & 2;
  const int z = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool zin = z < v;
  const int ny = (v - w + SW_NW - 1) / SW_NW;  // rows of this wave
  cplx a3[SW_MAXY], a5[SW_MAXY];
#pragma unroll
  for (int k = 0; k < SW_MAXY; ++k) {
    a3[k] = cplx{0, 0};
    a5[k] = cplx{0, 0};
  }
  cplx a4{0, 0};
  const cplx fz = zin ? fK[z] : cplx{0, 0};
  for (int x = xb; x < xe; ++x) {
    const cplx fx = fK[x];
    const cplx* tx = t + (int64_t)x * v2;
    cplx p1{0, 0}, p2{0, 0};
#pragma unroll
    for (int k = 0; k < SW_MAXY; ++k) {
      if (k < ny) {
        const int y = w + SW_NW * k;
        const cplx tv = zin ? tx[(int64_t)y * v + z] : cplx{0, 0};
        if (doX) {
          if (zin) {
            p1 = cadd(p1, cmul(tv, LJ[y * Ly + z]));
            a3[k] = cadd(a3[k], cmul(tv, fx));
            a4 = cadd(a4, cmul(tv, LJ[y * Ly + x]));
          }
          // X2a[x][y] = sum_z t[x,y,z] f[z]: wave reduction over the lanes
          cplx r = cmul(tv, fz);
          for (int off = 32; off > 0; off >>= 1) {
            r.re += __shfl_xor(r.re, off);
            r.im += __shfl_xor(r.im, off);
          }
          if (z == 0) catomic(&X2p[(((int64_t)I * o + J) * v + x) * v + y], r);
        }
        if (doZ && zin) {
          p2 = cadd(p2, cmul(tv, l2JK[(int64_t)y * v + z]));
          a5[k] = cadd(a5[k], cmul(tv, l2JK[(int64_t)x * v + z]));
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      p1.re += __shfl_xor(p1.re, off);
      p1.im += __shfl_xor(p1.im, off);
      p2.re += __shfl_xor(p2.re, off);
      p2.im += __shfl_xor(p2.im, off);
    }
    if (z == 0) {
      sx[0][w][x] = p1;
      sx[1][w][x] = p2;
    }
  }
  // X2b[z][y] = sum_x t[x,y,z] f[x] (subtracted); Zb[y] = sum_xz t l2[x][z] (subtracted)
#pragma unroll
  for (int k = 0; k < SW_MAXY; ++k) {
    if (k < ny) {
      const int y = w + SW_NW * k;
      if (doX && zin) catomic(&X2p[(((int64_t)I * o + J) * v + z) * v + y], cplx{-a3[k].re, -a3[k].im});
      if (doZ) {
        cplx r = a5[k];
        for (int off = 32; off > 0; off >>= 1) {
          r.re += __shfl_xor(r.re, off);
          r.im += __shfl_xor(r.im, off);
        }
        if (z == 0) catomic(&Z[(int64_t)I * v + y], cplx{-r.re, -r.im});
      }
    }
  }
  sz[w][z] = a4;
  __syncthreads();
  if (threadIdx.x < v) {
    const int a = threadIdx.x;
    const bool own = a >= xb && a < xe;  // X1a[a] and Za[a] belong to this chunk
    cplx s1{0, 0}, s2{0, 0}, s4{0, 0};
    for (int ww = 0; ww < SW_NW; ++ww) {
      if (own) {
        s1 = cadd(s1, sx[0][ww][a]);
        s2 = cadd(s2, sx[1][ww][a]);
      }
      s4 = cadd(s4, sz[ww][a]);
    }
    if (doX) catomic(&X1[(int64_t)I * v + a], csub(s1, s4));
    if (doZ && own) catomic(&Z[(int64_t)I * v + a], s2);
  }
}

// Tiled P_ijk^abc + denominator for one canonical triple c = (i<=j<=k) per
// blockIdx.y, one 8x8x8 cube of (a,b,c) per blockIdx.x.  With p_s the six
// permutations (identity, (12), (23), (13), cyclic, cyclic^2) of positions,
//   t_c[t] = sum_s W[slot_s][t o p_s] / D(t),   T[slot_s][t o p_s] = t_c[t]
// where slot_s is the window slot of the ordered triple (i,j,k) o p_s, because
// t_{sigma(ijk)}^{sigma(abc)} = t_{ijk}^{abc}.  Sources are read and
// destinations written along their unit-stride index through LDS.
constexpr int CB = 8;
__device__ __constant__ int kPerm[6][3] = {{0, 1, 2}, {1, 0, 2}, {0, 2, 1}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}};

// With LAM, each source element first receives the terms of the lambda3 bracket
// that carry no summation index,
//   L_ijab l_c^k - L_ijac l_b^k + f~_ia l_bc^jk - f~_ja l_bc^ik,
// evaluated at that source's own occupied and virtual indices.
template <bool LAM>
__global__ __launch_bounds__(256) void sym_cube_kernel(const cplx* __restrict__ W, cplx* __restrict__ T,
                                                         const int* __restrict__ canon, const int* __restrict__ part,
                                                         const double* __restrict__ eps, int o, int v, LamElem le) {
  __shared__ cplx acc[CB * CB * CB];
  const int q = blockIdx.y;
  const int I = canon[4 * q], J = canon[4 * q + 1], K = canon[4 * q + 2], n0 = canon[4 * q + 3];
  const int* sl = part + 6 * n0;
  const int nc = (v + CB - 1) / CB;
  const int cube = blockIdx.x;
  int t0[3];
  t0[0] = (cube / (nc * nc)) * CB;
  t0[1] = ((cube / nc) % nc) * CB;
  t0[2] = (cube % nc) * CB;
  const int64_t v3 = (int64_t)v * v * v;
  for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) acc[e] = cplx{0, 0};
  __syncthreads();
  const int occ[3] = {I, J, K};
  const int nn = o + v;
  for (int s = 0; s < 6; ++s) {
    const int p0 = kPerm[s][0], p1 = kPerm[s][1], p2 = kPerm[s][2];
    const int x0 = t0[p0], x1 = t0[p1], x2 = t0[p2];
    const cplx* src = W + (int64_t)sl[s] * v3;
    const int si = occ[p0], sj = occ[p1], sk = occ[p2];  // the source's occupied triple
    for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
      const int u0 = e / (CB * CB), u1 = (e / CB) % CB, u2 = e % CB;
      const int X0 = x0 + u0, X1 = x1 + u1, X2 = x2 + u2;
      if (X0 < v && X1 < v && X2 < v) {
        int tl[3];
        tl[p0] = u0;
        tl[p1] = u1;
        tl[p2] = u2;
        cplx w = src[((int64_t)X0 * v + X1) * v + X2];
        if (LAM) {
          const cplx* Lij = le.Lov + (((int64_t)si * v + X0) * o + sj) * v;  // L[si,X0,sj,:]
          w = cadd(w, cmul(Lij[X1], le.l1[(int64_t)sk * v + X2]));
          w = csub(w, cmul(Lij[X2], le.l1[(int64_t)sk * v + X1]));
          w = cadd(w, cmul(le.F[(int64_t)si * nn + o + X0], le.l2[(((int64_t)sj * o + sk) * v + X1) * v + X2]));
          w = csub(w, cmul(le.F[(int64_t)sj * nn + o + X0], le.l2[(((int64_t)si * o + sk) * v + X1) * v + X2]));
        }
        cplx& r = acc[(tl[0] * CB + tl[1]) * CB + tl[2]];
        r.re += w.re;
        r.im += w.im;
      }
    }
    __syncthreads();
  }
  const double eocc = eps[I] + eps[J] + eps[K];
  for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
    const int a = t0[0] + e / (CB * CB), b = t0[1] + (e / CB) % CB, c = t0[2] + e % CB;
    if (a < v && b < v && c < v) {
      const double D = eocc - eps[o + a] - eps[o + b] - eps[o + c];
      acc[e].re /= D;
      acc[e].im /= D;
    }
  }
  __syncthreads();
  for (int s = 0; s < 6; ++s) {
    const int p0 = kPerm[s][0], p1 = kPerm[s][1], p2 = kPerm[s][2];
    const int x0 = t0[p0], x1 = t0[p1], x2 = t0[p2];
    cplx* dst = T + (int64_t)sl[s] * v3;
    for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
      const int u0 = e / (CB * CB), u1 = (e / CB) % CB, u2 = e % CB;
      const int X0 = x0 + u0, X1 = x1 + u1, X2 = x2 + u2;
      if (X0 < v && X1 < v && X2 < v) {
        int tl[3];
        tl[p0] = u0;
        tl[p1] = u1;
        tl[p2] = u2;
        dst[((int64_t)X0 * v + X1) * v + X2] = acc[(tl[0] * CB + tl[1]) * CB + tl[2]];
      }
    }
  }
}

}  // namespace

void launch_sym_cube(const cplx* W, cplx* T, const int* canon, int ncanon, const int* part, const double* eps, int o,
                     int v, const LamElem* le, hipStream_t s) {
  if (ncanon <= 0) return;
  const int nc = (v + CB - 1) / CB;
  const dim3 grid((unsigned)(nc * nc * nc), (unsigned)ncanon);
  if (le) {
    hipLaunchKernelGGL(sym_cube_kernel<true>, grid, dim3(256), 0, s, W, T, canon, part, eps, o, v, *le);
  } else {
    hipLaunchKernelGGL(sym_cube_kernel<false>, grid, dim3(256), 0, s, W, T, canon, part, eps, o, v, LamElem{});
  }
  RTCC3_HIP(hipGetLastError());
}

void launch_small_t3(const cplx* T, const int* bl, int nb, const cplx* Lov, const cplx* F, const cplx* l2, cplx* X1,
                     cplx* X2p, cplx* Z, int o, int v, int flags, hipStream_t s) {
  if (nb <= 0) return;
  if (v <= 64) {
    const unsigned nxc = (unsigned)((v + SW_XCHUNK - 1) / SW_XCHUNK);
    hipLaunchKernelGGL(small_t3_wave_kernel, dim3((unsigned)nb, nxc), dim3(64 * SW_NW), 0, s, T, bl, Lov, F, l2, X1, X2p,
                       Z, o, v, flags);
  } else {
    hipLaunchKernelGGL(small_t3_simple_kernel, dim3((unsigned)v, (unsigned)nb), dim3(64), 0, s, T, bl, Lov, F, l2, X1,
                       X2p, Z, o, v, flags);
  }
  RTCC3_HIP(hipGetLastError());
}

}  // namespace rtcc3
