// Device-side building blocks: complex arithmetic, small DFTs, an in-LDS Stockham FFT
// (self-sorting, radix 8/4/2 passes), real-FFT packing, and cubic B-spline weights.
#pragma once

#include <hip/hip_runtime.h>

namespace rl {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward, INV=false) or +i (inverse, INV=true)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// 3-point DFT: X_k = sum_j v_j w^{jk}, w = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2.
template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float h = 0.86602540378443864676f;  // sqrt(3) / 2
  const float2 t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
  const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
  // (-+ i) sqrt(3)/2 d
  const float2 s = INV ? make_float2(-h * d.y, h * d.x) : make_float2(h * d.y, -h * d.x);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, s);
  v[2] = csub(m, s);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // twiddles exp(-+ 2 pi i k / 8), k = 0..3
  float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                  : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = mul_mi<INV>(o[2]);
  float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                  : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else dft8<INV>(v);
}

// Twiddles of the Stockham passes, laid out per pass (built with the plan): the pass of
// radix R after sub-transforms of length Ns holds, for k = 0 .. Ns - 1, the R - 1 twiddles
// exp(-2 pi i r k / (R Ns)), r = 1 .. R - 1, padded to an even count (RP entries), so that
// a butterfly reads its twiddles as consecutive 16-byte loads.  Lengths 2^a 3^b take their
// radix-3 passes first, then radix 8, 4 and 2 as the power of two allows.
__host__ __device__ constexpr int stockham_radix(int left) {
  return left % 3 == 0 ? 3 : (left >= 8 ? 8 : (left == 4 ? 4 : 2));
}
__host__ __device__ constexpr int stockham_slots(int R) { return R == 8 ? 8 : (R == 4 ? 4 : 2); }

// One Stockham pass of radix R over nfft independent FFTs of length N stored back to back
// in LDS (buf[f*N + i]).  Ns is the length of the sub-transforms already done; twp points at
// this pass's twiddles.  Every thread of the block must call it (it contains barriers).
// MAXB bounds the butterflies per thread.
template <int R, int MAXB, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, int N, int nfft, int Ns, const float2* __restrict__ twp) {
  constexpr int RP = stockham_slots(R);
  const int nbf = N / R;
  const int total = nbf * nfft;
  float2 v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int id = threadIdx.x + b * blockDim.x;
    if (id < total) {
      const int f = id / nbf;
      const int j = id - f * nbf;
      const int k = (Ns & (Ns - 1)) == 0 ? (j & (Ns - 1)) : j % Ns;
      const float2* base = buf + f * N;
      float2 w[RP];
      if (Ns > 1) {  // uniform; the first pass multiplies by exp(0) = 1
        const float4* tq = reinterpret_cast<const float4*>(twp + k * RP);
#pragma unroll
        for (int i = 0; i < RP / 2; ++i) {
          const float4 t = tq[i];
          w[2 * i] = make_float2(t.x, t.y);
          w[2 * i + 1] = make_float2(t.z, t.w);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = base[j + r * nbf];
        if (r > 0 && Ns > 1) {
          float2 tw = w[r - 1];
          if (INV) tw.y = -tw.y;
          x = cmul(x, tw);
        }
        v[b][r] = x;
      }
      dft<R, INV>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int id = threadIdx.x + b * blockDim.x;
    if (id < total) {
      const int f = id / nbf;
      const int j = id - f * nbf;
      const int k = (Ns & (Ns - 1)) == 0 ? (j & (Ns - 1)) : j % Ns;
      float2* base = buf + f * N;
      const int o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) base[o + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

// Unnormalised in-place FFT (forward: exp(-2 pi i jk/N); INV: exp(+...)) of nfft
// transforms of length N = 2^a 3^b >= 2 held in LDS; twp is the pass twiddle table of
// length N.  MAXV bounds the complex values per thread: nfft * N <= MAXV * blockDim.x.
// Callers synchronise before the call.
template <int MAXV, bool INV>
__device__ __forceinline__ void fft_lds(float2* buf, int N, int nfft, const float2* __restrict__ twp) {
  int Ns = 1;
  while (Ns < N) {
    const int R = stockham_radix(N / Ns);
    if (R == 8) stockham_pass<8, MAXV / 8, INV>(buf, N, nfft, Ns, twp);
    else if (R == 4) stockham_pass<4, MAXV / 4, INV>(buf, N, nfft, Ns, twp);
    else if (R == 3) stockham_pass<3, (MAXV + 2) / 3, INV>(buf, N, nfft, Ns, twp);
    else stockham_pass<2, MAXV / 2, INV>(buf, N, nfft, Ns, twp);
    twp += Ns * stockham_slots(R);
    Ns *= R;
  }
}

// Values a thread handles per chunk in the row loops below.  A loop over a row with a global
// load per iteration would wait a full memory round trip per iteration (nothing lets the
// compiler overlap iterations of a loop whose trip count is unknown); these loops issue all
// loads of a chunk first, then consume them.  Fewer values per chunk (kChunkSmall) leave the
// registers for more waves; which is faster depends on the kernel (measured per kernel).
constexpr int kChunk = 8;
constexpr int kChunkSmall = 4;

// For i in [0, n), strided over the block: put(i, get(i)), the gets of a chunk of CH values
// per thread issued together (unconditionally: an index past the end reads entry n - 1,
// unused, so that no branch splits the loads).  n >= 1.
template <int CH = kChunk, class Get, class Put>
__device__ __forceinline__ void row_copy(int n, Get get, Put put) {
  using T = decltype(get(0));
  for (int base = 0; base < n; base += CH * (int)blockDim.x) {
    T v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = get(min(base + (int)threadIdx.x + c * (int)blockDim.x, n - 1));
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = base + (int)threadIdx.x + c * (int)blockDim.x;
      if (i < n) put(i, v[c]);
    }
  }
}

// Real FFT post-processing: Z = FFT_nc(x[2n] + i x[2n+1]) in LDS -> X[k], k = 0..nc, of the
// length-2nc real signal.  Calls fn(k, X[k]) for every k in [0, nc].  Threads stride over
// k in [0, nc/2]; each handles k and nc - k.
template <int CH = kChunk, class Fn>
__device__ __forceinline__ void rfft_post(const float2* Z, int nc, const float2* __restrict__ tw,
                                          int tw_len, Fn fn) {
  const int step = tw_len / (2 * nc);
  const int half = nc / 2;
  for (int base = 0; base <= half; base += CH * (int)blockDim.x) {
    float2 w1[CH], w2[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {  // twiddles of the chunk (global) first, unconditionally
      const int k = min(base + (int)threadIdx.x + c * (int)blockDim.x, half);
      w1[c] = tw[k * step];
      w2[c] = tw[(nc - k) * step];  // k = 0: exp(-i pi) = -1
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = base + (int)threadIdx.x + c * (int)blockDim.x;
      if (k > half) continue;
      const int km = nc - k;
      const float2 a = Z[k == 0 ? 0 : k];
      const float2 b = Z[k == 0 ? 0 : km];
      // X[k] = (a + conj b)/2 - i/2 w^k (a - conj b),  w = exp(-2 pi i / (2 nc))
      const float2 e = cscale(cadd(a, cconj(b)), 0.5f);
      const float2 o = cscale(csub(a, cconj(b)), 0.5f);
      const float2 t = cmul(w1[c], o);
      fn(k, make_float2(e.x + t.y, e.y - t.x));
      if (km != k) {
        // X[nc - k] from the same pair with roles swapped
        const float2 e2 = cscale(cadd(b, cconj(a)), 0.5f);
        const float2 o2 = cscale(csub(b, cconj(a)), 0.5f);
        const float2 t2 = cmul(km == nc ? make_float2(-1.f, 0.f) : w2[c], o2);
        fn(km, make_float2(e2.x + t2.y, e2.y - t2.x));
      }
    }
  }
}

// Inverse real FFT pre-processing: X[k], k = 0..nc (read through get(k)) -> Z[k], k < nc,
// such that the unnormalised inverse FFT_nc of Z gives z[n] = y[2n] + i y[2n+1] where y is
// the unnormalised inverse DFT of length 2nc of the Hermitian extension of X.
template <int CH = kChunk, class Get>
__device__ __forceinline__ void irfft_pre(float2* Z, int nc, const float2* __restrict__ tw,
                                          int tw_len, Get get) {
  const int step = tw_len / (2 * nc);
  for (int base = 0; base < nc; base += CH * (int)blockDim.x) {
    float2 xa[CH], xb[CH], w[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {  // every load of the chunk first, unconditionally
      const int k = min(base + (int)threadIdx.x + c * (int)blockDim.x, nc - 1);
      xa[c] = get(k);
      xb[c] = get(nc - k);
      w[c] = tw[k * step];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = base + (int)threadIdx.x + c * (int)blockDim.x;
      if (k >= nc) continue;
      const float2 a = xa[c];
      const float2 b = cconj(xb[c]);
      const float2 e = cadd(a, b);
      const float2 d = csub(a, b);
      const float2 wc = cconj(w[c]);  // exp(+2 pi i k / (2 nc))
      const float2 o = cmul(d, wc);
      Z[k] = make_float2(e.x - o.y, e.y + o.x);  // e + i o
    }
  }
}

// In-register FFT of compile-time length R = 2^a 3^b.  Unnormalised; forward uses
// exp(-2 pi i jk/R), INV the conjugate.  Twiddles are read from the plan's table
// tw[n] = exp(-2 pi i n / tw_len) (tw_len a multiple of R).  A factor 3 is split off first
// (decimation in time: three interleaved sub-transforms of length R/3, then radix-3
// butterflies with twiddles w^{s k}); a power of two runs radix-2 decimation in time with a
// compile-time bit reversal, the twiddles 1 and -i (+i inverse) applied without a multiply.
template <int R>
constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1, j = R >> 1; b < R; b <<= 1, j >>= 1)
    if (i & b) r |= j;
  return r;
}

template <int R, bool INV>
__device__ __forceinline__ void reg_fft(float2 (&v)[R], const float2* __restrict__ tw, int tw_len) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R % 3 == 0) {
    constexpr int R3 = R / 3;
    float2 sub[3][R3];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int j = 0; j < R3; ++j) sub[s][j] = v[3 * j + s];
#pragma unroll
    for (int s = 0; s < 3; ++s) reg_fft<R3, INV>(sub[s], tw, tw_len);
    const int tstep = tw_len / R;
#pragma unroll
    for (int k = 0; k < R3; ++k) {
      float2 x[3];
      x[0] = sub[0][k];
#pragma unroll
      for (int s = 1; s < 3; ++s) {
        if (k == 0) {
          x[s] = sub[s][k];
        } else {
          float2 w = tw[s * k * tstep];
          if (INV) w.y = -w.y;
          x[s] = cmul(sub[s][k], w);
        }
      }
      dft3<INV>(x);
#pragma unroll
      for (int m = 0; m < 3; ++m) v[k + m * R3] = x[m];
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = bitrev<R>(i);
      if (i < j) {
        const float2 t = v[i];
        v[i] = v[j];
        v[j] = t;
      }
    }
    const int tstep = tw_len / R;
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
      const int half = len >> 1;
#pragma unroll
      for (int k = 0; k < half; ++k) {
        const int e = k * (R / len);  // exponent in units of 1/R turns
        float2 w;
        if (e == 0 || 4 * e == R) {  // 1 and -i (+i inverse) need no multiply
          w = make_float2(1.f, 0.f);
        } else {
          w = tw[e * tstep];
          if (INV) w.y = -w.y;
        }
#pragma unroll
        for (int i = 0; i < R; i += len) {
          const float2 a = v[i + k];
          const float2 b = (e == 0) ? v[i + k + half] : (4 * e == R) ? mul_mi<INV>(v[i + k + half]) : cmul(v[i + k + half], w);
          v[i + k] = cadd(a, b);
          v[i + k + half] = csub(a, b);
        }
      }
    }
  }
}

// Six times the cubic B-spline weights for taps k-1, k, k+1, k+2 at fractional offset a in
// [0, 1) (the factor 1/6 per dimension is applied once to the value instead).
__device__ __forceinline__ void bspline_w6(float a, float* w) {
  const float a2 = a * a, a3 = a2 * a;
  const float b = 1.0f - a;
  w[0] = b * b * b;
  w[1] = fmaf(3.0f, a3, fmaf(-6.0f, a2, 4.0f));
  w[2] = fmaf(-3.0f, a3, fmaf(3.0f, a2, fmaf(3.0f, a, 1.0f)));
  w[3] = a3;
}

// Image node (ix, iy) lies strictly inside the unit disc: its coordinates are (2i - n)/n, so the
// test is exact in integers (floating point could round nodes with |x| = 1 either way).
__device__ __forceinline__ bool in_unit_disc(int ix, int iy, int n) {
  const long long a = 2LL * ix - n, b = 2LL * iy - n;
  return a * a + b * b < (long long)n * n;
}

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Blocks are dispatched to the chip's 8 XCDs (each with its own L2) round-robin by linear
// block id.  xcd_block maps a linear id to a logical block such that every XCD gets one
// contiguous run of logical blocks: neighbouring blocks, which share cache lines, then run
// on the same XCD, one after the other.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int id, int nblocks) {
  const int xcd = id % kXcds, local = id / kXcds;
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  return xcd * per + min(xcd, rem) + local;
}

}  // namespace rl
