// Element-wise and reduction kernels of the triples engine (one block of
// [v,v,v] per ordered occupied triple n, row-major [a][b][c]).
#include "triples_kernels.h"

#include <algorithm>

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

// Contractions with one free virtual index per block (I,J,K):
//   flags&1: X1[I][a]     += sum_bc (t[a,b,c] - t[c,b,a]) L[J,b,K,c]
//            X2p[I,J][a,b]+= sum_c  (t[a,b,c] - t[c,b,a]) f~[K, c]
//   flags&2: Z[I][a]      += sum_bc (t[a,b,c] - t[b,a,c]) l2[J,K,b,c]
// One (block, a) per workgroup; used when v > 128 (the wave kernel below maps
// the unit-stride index onto the 64 lanes of a wave, in up to two chunks).
__global__ void small_t3_simple_kernel(const cplx* __restrict__ T, const int* __restrict__ bl, const cplx* __restrict__ Lov,
                                const cplx* __restrict__ F, const cplx* __restrict__ l2, cplx* __restrict__ X1,
                                cplx* __restrict__ X2p, cplx* __restrict__ Z, int o, int v, int vp, int flags) {
  const int q = blockIdx.y, a = blockIdx.x;
  const int I = bl[4 * q], J = bl[4 * q + 1], K = bl[4 * q + 2], n = bl[4 * q + 3];
  const int64_t va = (int64_t)v * vp, vb = va * v;  // padded block strides
  const int nn = o + v;
  const cplx* t = T + (int64_t)n * vb;
  cplx x1{0, 0}, z{0, 0};
  for (int b = threadIdx.x; b < v; b += blockDim.x) {
    cplx x2f{0, 0};
    const cplx* Lb = Lov + (((int64_t)J * v + b) * o + K) * v;
    const cplx* l2b = l2 + (((int64_t)J * o + K) * v + b) * v;
    for (int c = 0; c < v; ++c) {
      const cplx tabc = t[a * va + (int64_t)b * vp + c];
      if (flags & 1) {
        const cplx tz = csub(tabc, t[c * va + (int64_t)b * vp + a]);
        x1 = cadd(x1, cmul(tz, Lb[c]));
        x2f = cadd(x2f, cmul(tz, F[(int64_t)K * nn + o + c]));
      }
      if (flags & 2) z = cadd(z, cmul(csub(tabc, t[b * va + (int64_t)a * vp + c]), l2b[c]));
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

// Sum of eight values over the 64 lanes of a wave: on return lane l holds in
// v[0] the total of v[l >> 3] (reduce-scatter by halving, then the last three
// lane bits), ten complex exchanges instead of eight full reductions.
__device__ __forceinline__ void wave_sum8(cplx* v, int lane) {
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  auto xch = [](cplx x, int m) { return cplx{__shfl_xor(x.re, m), __shfl_xor(x.im, m)}; };
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const cplx mine = h5 ? v[4 + j] : v[j], other = h5 ? v[j] : v[4 + j];
    v[j] = cadd(mine, xch(other, 32));
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const cplx mine = h4 ? v[2 + j] : v[j], other = h4 ? v[j] : v[2 + j];
    v[j] = cadd(mine, xch(other, 16));
  }
  {
    const cplx mine = h3 ? v[1] : v[0], other = h3 ? v[0] : v[1];
    v[0] = cadd(mine, xch(other, 8));
  }
  v[0] = cadd(v[0], xch(v[0], 4));
  v[0] = cadd(v[0], xch(v[0], 2));
  v[0] = cadd(v[0], xch(v[0], 1));
}

// One workgroup of SW_NW waves per block and chunk of SW_NW rows y
// (blockIdx.y); wave w owns the row y = SW_NW*chunk + w, lane = z within each
// of NZC 64-wide chunks of the unit-stride index (v <= 64 NZC), and the wave
// walks x four at a time (fewer live registers, so the kernel shares the chip
// with the products that run beside it).  Every element of a block is read
// once, as part of a coalesced row.  Sums over z use wave_sum8 on the terms of
// four x at once (after adding the z chunks); sums over x stay in registers,
// per z chunk, so X2b and Zb are complete per workgroup; X1a, Za, X1b (sums
// over y) go through LDS and are added per chunk of rows.
constexpr int SW_NW = 8;

template <int NZC>
__global__ __launch_bounds__(64 * SW_NW) void small_t3_wave_kernel(const cplx* __restrict__ T, const int* __restrict__ bl,
                                                              const cplx* __restrict__ Lov, const cplx* __restrict__ F,
                                                              const cplx* __restrict__ l2, cplx* __restrict__ X1,
                                                              cplx* __restrict__ X2p, cplx* __restrict__ Z, int o,
                                                              int v, int vp, int flags) {
  constexpr int VZ = 64 * NZC;
  __shared__ cplx sP[2][SW_NW][VZ];  // per-wave X1a[x], Za[x]
  __shared__ cplx sz[SW_NW][VZ];     // per-wave X1b[z]
  const int q = blockIdx.x;
  const int I = bl[4 * q], J = bl[4 * q + 1], K = bl[4 * q + 2], n = bl[4 * q + 3];
  const int64_t v2 = (int64_t)v * v, va = (int64_t)v * vp;  // t[x][y][z] at x*va + y*vp + z
  const int nn = o + v;
  const cplx* t = T + (int64_t)n * va * v;
  const cplx* fK = F + (int64_t)K * nn + o;
  const cplx* l2JK = l2 + ((int64_t)J * o + K) * v2;
  const int64_t Ly = (int64_t)o * v;
  const bool doX = flags & 1, doZ = flags & 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int y = blockIdx.y * SW_NW + w;
  const bool yin = y < v;
  const cplx* LJy = Lov + (int64_t)J * v * o * v + (int64_t)K * v + (yin ? y * Ly : 0);  // L[J,y,K,.]
  bool zin[NZC];
  cplx Lyz[NZC], lyz[NZC], fz[NZC], a3[NZC], a4[NZC];
#pragma unroll
  for (int c = 0; c < NZC; ++c) {
    const int z = 64 * c + lane;
    zin[c] = z < v;
    const bool ok = yin && zin[c];
    Lyz[c] = ok ? LJy[z] : cplx{0, 0};
    lyz[c] = ok ? l2JK[(int64_t)y * v + z] : cplx{0, 0};
    fz[c] = zin[c] ? fK[z] : cplx{0, 0};
    a3[c] = a4[c] = cplx{0, 0};
  }
  cplx a5{0, 0};
  for (int xg = 0; xg < v; xg += 4) {
    // four x at a time: u = (X2a terms, X1a terms), zq = (Za terms, unused)
    cplx u[8], zq[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) u[e] = zq[e] = cplx{0, 0};
#pragma unroll
    for (int xl = 0; xl < 4; ++xl) {
      const int x = xg + xl;
      const bool xin = x < v;
      const cplx fx = xin ? fK[x] : cplx{0, 0};
      const cplx Lx = xin && yin ? LJy[x] : cplx{0, 0};
#pragma unroll
      for (int c = 0; c < NZC; ++c) {
        const int z = 64 * c + lane;
        const bool ok = yin && zin[c] && xin;
        const cplx tv = ok ? t[(int64_t)x * va + (int64_t)y * vp + z] : cplx{0, 0};
        u[xl] = cadd(u[xl], cmul(tv, fz[c]));
        u[4 + xl] = cadd(u[4 + xl], cmul(tv, Lyz[c]));
        zq[xl] = cadd(zq[xl], cmul(tv, lyz[c]));
        a3[c] = cadd(a3[c], cmul(tv, fx));
        a4[c] = cadd(a4[c], cmul(tv, Lx));
        a5 = cadd(a5, cmul(tv, zin[c] && xin ? l2JK[(int64_t)x * v + z] : cplx{0, 0}));
      }
    }
    const int qi = lane >> 3;                   // the entry a lane's reduced value belongs to
    const int xs = xg + (qi & 3);               // ... and its x
    if (doX) {
      // X2a[x][y] = sum_z t[x,y,z] f[z] (entries 0..3), X1a[x] per row (entries 4..7)
      wave_sum8(u, lane);
      if ((lane & 7) == 0 && xs < v) {
        if (qi < 4) {
          if (yin) catomic(&X2p[(((int64_t)I * o + J) * v + xs) * v + y], u[0]);
        } else {
          sP[0][w][xs] = u[0];
        }
      }
    }
    if (doZ) {
      wave_sum8(zq, lane);
      if ((lane & 7) == 0 && qi < 4 && xs < v) sP[1][w][xs] = zq[0];
    }
  }
#pragma unroll
  for (int c = 0; c < NZC; ++c) {
    const int z = 64 * c + lane;
    // X2b[z][y] = sum_x t[x,y,z] f[x] (subtracted)
    if (doX && yin && zin[c]) catomic(&X2p[(((int64_t)I * o + J) * v + z) * v + y], cplx{-a3[c].re, -a3[c].im});
    sz[w][z] = a4[c];
  }
  if (doZ) {  // Zb[y] = sum_xz t l2[x][z] (subtracted)
    for (int off = 32; off > 0; off >>= 1) {
      a5.re += __shfl_xor(a5.re, off);
      a5.im += __shfl_xor(a5.im, off);
    }
    if (lane == 0 && yin) catomic(&Z[(int64_t)I * v + y], cplx{-a5.re, -a5.im});
  }
  __syncthreads();
  for (int a = threadIdx.x; a < v; a += blockDim.x) {
    const int nw = min(SW_NW, v - (int)blockIdx.y * SW_NW);  // waves with a row
    cplx s1{0, 0}, s2{0, 0}, s4{0, 0};
    for (int ww = 0; ww < nw; ++ww) {
      if (doX) s1 = cadd(s1, sP[0][ww][a]);
      if (doZ) s2 = cadd(s2, sP[1][ww][a]);
      s4 = cadd(s4, sz[ww][a]);
    }
    if (doX) catomic(&X1[(int64_t)I * v + a], csub(s1, s4));
    if (doZ) catomic(&Z[(int64_t)I * v + a], s2);
  }
}

// Tiled P_ijk^abc + denominator for one canonical triple c = (i<=j<=k) per
// blockIdx.y, one 8x8x8 cube of (a,b,c) per blockIdx.x, in place.  With p_s
// the six permutations (identity, (12), (23), (13), cyclic, cyclic^2) of
// positions,
//   t_c[t] = sum_s W[slot_s][t o p_s] / D(t),   W[slot_s][t o p_s] <- t_c[t]
// where slot_s is the window slot of the ordered triple (i,j,k) o p_s, because
// t_{sigma(ijk)}^{sigma(abc)} = t_{ijk}^{abc}.  A workgroup reads the six
// (slot, cube) places it writes, all of them before any write, and the places
// of different workgroups are disjoint: for distinct i, j, k the six slots
// differ; when two occupied indices coincide, two slots are one block and the
// cubes related by swapping the matching virtual positions form one set of
// places, handled by the workgroup of the cube whose coordinates are ordered
// there (the others return at once).  Sources are read and destinations
// written along their unit-stride index through LDS.  The LDS cube is padded
// (row strides CB+1 and CB*(CB+1)+1 elements, both odd) so that walking any of
// its three axes touches distinct banks.
constexpr int CB = 8;
constexpr int CS1 = CB + 1, CS0 = CB * CS1 + 1;
__device__ __forceinline__ int cube_at(int t0, int t1, int t2) { return t0 * CS0 + t1 * CS1 + t2; }
// LDS stride of cube axis p: an element whose source coordinates u_k lie on
// cube axes p_k sits at sum_k u_k * cstride(p_k)
__device__ __forceinline__ int cstride(int p) { return p == 0 ? CS0 : p == 1 ? CS1 : 1; }
__device__ __constant__ int kPerm[6][3] = {{0, 1, 2}, {1, 0, 2}, {0, 2, 1}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}};

// With NL > 0, each source element first receives the terms of the lambda3
// bracket that carry no summation index,
//   L_ijab l_c^k - L_ijac l_b^k + f~_ia l_bc^jk - f~_ja l_bc^ik,
// evaluated at that source's own occupied and virtual indices, from NL sets of
// inputs (a null input of a set reads as zero; the derivative of the terms
// takes two sets, e.g. (L, f~', l1', l2) and (f~, l2')).
struct LamPair {
  LamElem e[2];
};
template <int NL>
__global__ __launch_bounds__(256) void sym_cube_kernel(cplx* __restrict__ W, const int* __restrict__ canon,
                                                         const int* __restrict__ part,
                                                         const double* __restrict__ eps, int o, int v, int vp,
                                                         LamPair le) {
  __shared__ cplx acc[CB * CS0];
  const int q = blockIdx.y;
  const int I = canon[4 * q], J = canon[4 * q + 1], K = canon[4 * q + 2], n0 = canon[4 * q + 3];
  const int* sl = part + 6 * n0;
  const int nc = (v + CB - 1) / CB;
  const int cube = blockIdx.x;
  const int q0 = cube / (nc * nc), q1 = (cube / nc) % nc, q2 = cube % nc;
  if ((I == J && q0 > q1) || (J == K && q1 > q2)) return;  // another workgroup owns these places
  const int c0 = q0 * CB, c1 = q1 * CB, c2 = q2 * CB;  // cube corner
  // (selects rather than arrays indexed by the permutation, which would live in scratch memory)
  auto pick = [](int p, int a, int b, int c) { return p == 0 ? a : p == 1 ? b : c; };
  const int64_t vb = (int64_t)v * v * vp;  // block stride; element [X0][X1][X2] at (X0*v + X1)*vp + X2
  for (int e = threadIdx.x; e < CB * CS0; e += blockDim.x) acc[e] = cplx{0, 0};
  __syncthreads();
  const int nn = o + v;
  // With NL > 0, a source's terms without a summation index need, per cube and
  // set, only 8x8 slices of L and l2 and 8-vectors of l1 and f~: staged in LDS first.
  constexpr int NS = NL > 0 ? NL : 1;
  __shared__ cplx lt[NS][4][CB][CB];  // L[si,X0,sj,X1], L[si,X0,sj,X2], l2[sj,sk,X1,X2], l2[si,sk,X1,X2]
  __shared__ cplx lv[NS][4][CB];      // l1[sk,X2], l1[sk,X1], f~[si,X0], f~[sj,X0]
  for (int s = 0; s < 6; ++s) {
    const int p0 = kPerm[s][0], p1 = kPerm[s][1], p2 = kPerm[s][2];
    const int x0 = pick(p0, c0, c1, c2), x1 = pick(p1, c0, c1, c2), x2 = pick(p2, c0, c1, c2);
    const cplx* src = W + (int64_t)sl[s] * vb;
    const int si = pick(p0, I, J, K), sj = pick(p1, I, J, K), sk = pick(p2, I, J, K);  // the source's occupied triple
    if (NL > 0) {
      static_assert(CB == 8, "the staging below maps 256 threads onto four 8x8 tables");
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const LamElem& ler = le.e[r];
        const int tq = threadIdx.x >> 6, i = (threadIdx.x >> 3) & 7, j = threadIdx.x & 7;
        // table tq, row i, column j: one pointer and one range test per thread
        const int ri = tq < 2 ? x0 : x1, cj = tq == 0 ? x1 : x2;  // virtual offsets of the row and column
        const cplx* tb = tq < 2    ? (ler.Lov ? ler.Lov + ((int64_t)si * v * o + sj) * v : nullptr)  // L[si, ., sj, .]
                         : tq == 2 ? (ler.l2 ? ler.l2 + ((int64_t)sj * o + sk) * v * v : nullptr)    // l2[sj, sk, ., .]
                                   : (ler.l2 ? ler.l2 + ((int64_t)si * o + sk) * v * v : nullptr);   // l2[si, sk, ., .]
        const int64_t rs = tq < 2 ? (int64_t)o * v : v;  // row stride
        const bool okt = tb && ri + i < v && cj + j < v;
        lt[r][tq][i][j] = okt ? tb[(int64_t)(ri + i) * rs + cj + j] : cplx{0, 0};
        if (threadIdx.x < 4 * CB) {
          const int rr = threadIdx.x >> 3;
          const int off = rr == 0 ? x2 : rr == 1 ? x1 : x0;
          const cplx* vq = rr == 0   ? (ler.l1 ? ler.l1 + (int64_t)sk * v + x2 : nullptr)
                           : rr == 1 ? (ler.l1 ? ler.l1 + (int64_t)sk * v + x1 : nullptr)
                           : rr == 2 ? (ler.F ? ler.F + (int64_t)si * nn + o + x0 : nullptr)
                                     : (ler.F ? ler.F + (int64_t)sj * nn + o + x0 : nullptr);
          const bool okv = vq && off + j < v;
          lv[r][rr][j] = okv ? vq[j] : cplx{0, 0};
        }
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
      const int u0 = e / (CB * CB), u1 = (e / CB) % CB, u2 = e % CB;
      const int X0 = x0 + u0, X1 = x1 + u1, X2 = x2 + u2;
      if (X0 < v && X1 < v && X2 < v) {
        cplx w = src[((int64_t)X0 * v + X1) * vp + X2];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
          //   L_ijab l_c^k - L_ijac l_b^k + f~_ia l_bc^jk - f~_ja l_bc^ik at the source's indices
          w = cadd(w, cmul(lt[r][0][u0][u1], lv[r][0][u2]));
          w = csub(w, cmul(lt[r][1][u0][u2], lv[r][1][u1]));
          w = cadd(w, cmul(lv[r][2][u0], lt[r][2][u1][u2]));
          w = csub(w, cmul(lv[r][3][u0], lt[r][3][u1][u2]));
        }
        cplx& r = acc[u0 * cstride(p0) + u1 * cstride(p1) + u2 * cstride(p2)];
        r.re += w.re;
        r.im += w.im;
      }
    }
    __syncthreads();
  }
  const double eocc = eps[I] + eps[J] + eps[K];
  for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
    const int u0 = e / (CB * CB), u1 = (e / CB) % CB, u2 = e % CB;
    const int a = c0 + u0, b = c1 + u1, c = c2 + u2;
    if (a < v && b < v && c < v) {
      const double D = eocc - eps[o + a] - eps[o + b] - eps[o + c];
      cplx& r = acc[cube_at(u0, u1, u2)];
      r.re /= D;
      r.im /= D;
    }
  }
  __syncthreads();
  for (int s = 0; s < 6; ++s) {
    const int p0 = kPerm[s][0], p1 = kPerm[s][1], p2 = kPerm[s][2];
    const int x0 = pick(p0, c0, c1, c2), x1 = pick(p1, c0, c1, c2), x2 = pick(p2, c0, c1, c2);
    cplx* dst = W + (int64_t)sl[s] * vb;
    for (int e = threadIdx.x; e < CB * CB * CB; e += blockDim.x) {
      const int u0 = e / (CB * CB), u1 = (e / CB) % CB, u2 = e % CB;
      const int X0 = x0 + u0, X1 = x1 + u1, X2 = x2 + u2;
      if (X0 < v && X1 < v && X2 < v)
        dst[((int64_t)X0 * v + X1) * vp + X2] = acc[u0 * cstride(p0) + u1 * cstride(p1) + u2 * cstride(p2)];
    }
  }
}


// Gram product of the density's slabs:
//   D[i][j] += alpha * sum_s sum_k A[(slot_s + i) K + k] B[(slot_s + j) K + k],  i, j < o <= 16,
// one slab s per blockIdx.y and one K range per blockIdx.x.  A 16x16 output
// needs one MFMA block, so the four waves split K instead of the output: each
// stage puts 64 k of the o rows of both operands in LDS (a wave reads one
// row's 64 consecutive elements), and wave w takes k in [16w, 16w + 16) of it.
// The four partial sums are added through LDS and the result with atomics.
constexpr int GR_KC = 64;
typedef double gr_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gram_kernel(const cplx* __restrict__ A, const cplx* __restrict__ B,
                                                   const int* __restrict__ slabs, int o, int64_t K, int64_t kchunk,
                                                   cplx alpha, cplx* __restrict__ D) {
  __shared__ double sm[2][2][16][GR_KC + 1];  // [A, B][re, im][row][k]
  const int64_t slot = slabs[4 * blockIdx.y + 3];
  const int64_t k0 = (int64_t)blockIdx.x * kchunk, k1 = min(K, k0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  gr_d4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
  // the next stage's elements are loaded into registers while the MFMAs of
  // the current one run
  cplx ra[4], rb[4];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r, row = e / GR_KC, c = e % GR_KC;
      const bool ok = row < o && kb + c < k1;
      const int64_t off = ok ? (slot + row) * K + kb + c : 0;
      ra[r] = ok ? A[off] : cplx{0, 0};
      rb[r] = ok ? B[off] : cplx{0, 0};
    }
  };
  load(k0);
  for (int64_t kb = k0; kb < k1; kb += GR_KC) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r, row = e / GR_KC, c = e % GR_KC;
      sm[0][0][row][c] = ra[r].re;
      sm[0][1][row][c] = ra[r].im;
      sm[1][0][row][c] = rb[r].re;
      sm[1][1][row][c] = rb[r].im;
    }
    __syncthreads();
    if (kb + GR_KC < k1) load(kb + GR_KC);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // lane l holds A[l%16][k] and, for B^T, B[l%16][k] with k = 16w + 4s + l/16
      const int m = lane & 15, kk = 16 * w + 4 * s + (lane >> 4);
      const double ar = sm[0][0][m][kk], ai = sm[0][1][m][kk];
      const double br = sm[1][0][m][kk], bi = sm[1][1][m][kk];
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, cim, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, cim, 0, 0, 0);
    }
    __syncthreads();
  }
  // partial sums of the four waves: result element [4r + l/16][l%16] of register r
  double* red = &sm[0][0][0][0];  // [wave][re, im][16][16], 16 KB of the 33 KB
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * r + (lane >> 4), j = lane & 15;
    red[((w * 2 + 0) * 16 + i) * 16 + j] = cre[r];
    red[((w * 2 + 1) * 16 + i) * 16 + j] = cim[r];
  }
  __syncthreads();
  const int i = tid >> 4, j = tid & 15;
  if (i < o && j < o) {
    double xr = 0, xi = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      xr += red[((ww * 2 + 0) * 16 + i) * 16 + j];
      xi += red[((ww * 2 + 1) * 16 + i) * 16 + j];
    }
    catomic(&D[i * o + j], cplx{alpha.re * xr - alpha.im * xi, alpha.re * xi + alpha.im * xr});
  }
}
}  // namespace

void launch_sym_cube(cplx* W, const int* canon, int ncanon, const int* part, const double* eps, int o, int v, int vp,
                     const LamElem* le, const LamElem* le2, hipStream_t s) {
  RTCC3_CHECK(vp >= v, "sym: row stride below v");
  RTCC3_CHECK(le || !le2, "sym: a second set of bracket inputs needs a first");
  if (ncanon <= 0) return;
  const int nc = (v + CB - 1) / CB;
  const dim3 grid((unsigned)(nc * nc * nc), (unsigned)ncanon);
  LamPair lp;
  if (le) lp.e[0] = *le;
  if (le2) lp.e[1] = *le2;
  if (le2)
    hipLaunchKernelGGL(sym_cube_kernel<2>, grid, dim3(256), 0, s, W, canon, part, eps, o, v, vp, lp);
  else if (le)
    hipLaunchKernelGGL(sym_cube_kernel<1>, grid, dim3(256), 0, s, W, canon, part, eps, o, v, vp, lp);
  else
    hipLaunchKernelGGL(sym_cube_kernel<0>, grid, dim3(256), 0, s, W, canon, part, eps, o, v, vp, lp);
  RTCC3_HIP(hipGetLastError());
}

void launch_gram(const cplx* A, const cplx* B, const int* slabs, int nslab, int o, int64_t K, cplx alpha, cplx* D,
                 hipStream_t s) {
  if (nslab <= 0 || K <= 0) return;
  RTCC3_CHECK(o >= 1 && o <= 16, "gram: at most 16 rows");
  // about 2048 workgroups over the slabs, K ranges in whole LDS stages
  const int64_t per = std::max<int64_t>(1, (2048 + nslab - 1) / nslab);
  const int64_t kchunk = ((K + per - 1) / per + GR_KC - 1) / GR_KC * GR_KC;
  const unsigned nx = (unsigned)((K + kchunk - 1) / kchunk);
  RTCC3_CHECK(nslab < 65536, "gram: too many slabs");
  hipLaunchKernelGGL(gram_kernel, dim3(nx, (unsigned)nslab), dim3(256), 0, s, A, B, slabs, o, K, kchunk, alpha, D);
  RTCC3_HIP(hipGetLastError());
}

void launch_small_t3(const cplx* T, const int* bl, int nb, const cplx* Lov, const cplx* F, const cplx* l2, cplx* X1,
                     cplx* X2p, cplx* Z, int o, int v, int vp, int flags, hipStream_t s) {
  RTCC3_CHECK(vp >= v, "small_t3: row stride below v");
  if (nb <= 0) return;
  const unsigned nyc = (unsigned)((v + SW_NW - 1) / SW_NW);
  if (v <= 64) {
    hipLaunchKernelGGL(small_t3_wave_kernel<1>, dim3((unsigned)nb, nyc), dim3(64 * SW_NW), 0, s, T, bl, Lov, F, l2, X1,
                       X2p, Z, o, v, vp, flags);
  } else if (v <= 128) {
    hipLaunchKernelGGL(small_t3_wave_kernel<2>, dim3((unsigned)nb, nyc), dim3(64 * SW_NW), 0, s, T, bl, Lov, F, l2, X1,
                       X2p, Z, o, v, vp, flags);
  } else {
    hipLaunchKernelGGL(small_t3_simple_kernel, dim3((unsigned)v, (unsigned)nb), dim3(64), 0, s, T, bl, Lov, F, l2, X1,
                       X2p, Z, o, v, vp, flags);
  }
  RTCC3_HIP(hipGetLastError());
}

}  // namespace rtcc3
