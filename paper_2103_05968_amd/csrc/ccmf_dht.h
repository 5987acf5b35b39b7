// Spectral solve of the periodic discrete Laplacian div^- grad^+ (the
// pseudo-inverse in eq:CCMF_FFT_Gamma_2) on the device.
//
// The Laplacian's symbol lambda(q) = -sum_c 4 sin^2(pi q_c / N_c) is real and
// even in every q_c separately, so the separable (per-axis) discrete Hartley
// transform H = H_1 (x) H_2 (x) H_3 diagonalises it with the same eigenvalues:
// every product of cos/sin modes along the three axes is an eigenvector.  Since
// H_c H_c = N_c Id, the solve is
//     phi = H (m . H r),   m(q) = 1 / (lambda(q) N),  m(0) = 0,
// i.e. five real-to-real passes: Hartley along k, along j, [along i, scale by m,
// along i] fused in one pass, along j, along k.  Each pass reads and writes one
// real field; no half-spectrum layout, no complex storage in HBM.
//
// A pass loads a tile of `nl` lines of length n into LDS, pairs lines a, b into
// one complex line a + i b, runs a mixed-radix Stockham FFT (radix 8, 4, 2 with
// fixed butterflies, any other radix with a direct DFT), and separates the two
// Hartley transforms:  with Z = FFT(a + i b) and Zm[q] = Z[-q],
//     H_a = (Re Z + Re Zm)/2 - (Im Z - Im Zm)/2,
//     H_b = (Im Z + Im Zm)/2 + (Re Z - Re Zm)/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccmf_kernels.h"

namespace ccmf {

constexpr int kMaxStages = 16;

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) { return {a.y, -a.x}; }  // -i a
template <typename T>
__device__ __forceinline__ C2<T> mul_pi(C2<T> a) { return {-a.y, a.x}; }  // +i a

struct DhtArgs {
  int32_t n;            // transform length
  int32_t nstages;
  int32_t radix[kMaxStages];
  int32_t nl;           // lines per tile (even)
  int32_t lines_total;  // lines along the tile's line dimension
  int32_t tiles_per_outer;
  int64_t ss;           // sample stride (elements)
  int64_t ls;           // line stride
  int64_t os;           // outer stride
  int64_t field_stride; // elements per field
  // spectral scaling of the fused middle pass
  double scale;         // 1/N
  int32_t n2, n3;       // sizes of the other two axes (middle pass: line index = q3, outer = q2)
};

// forward DFT of radix R on registers, exp(-2 pi i p r / R)
template <typename T>
__device__ __forceinline__ void dft2(C2<T>* v) {
  const C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T>* v) {
  const C2<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  const C2<T> a2 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, mul_mi(a3));
  v[3] = cadd(a1, mul_pi(a3));
}

template <typename T>
__device__ __forceinline__ void dft8(C2<T>* v) {
  C2<T> e[4] = {v[0], v[2], v[4], v[6]};
  C2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  const T h = T(0.70710678118654752440);
  // o[p] *= W8^p
  o[1] = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
  o[2] = mul_mi(o[2]);
  o[3] = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    v[p] = cadd(e[p], o[p]);
    v[p + 4] = csub(e[p], o[p]);
  }
}

// one Stockham stage with a fixed radix R in {2, 4, 8}
template <typename T, int R>
__device__ __forceinline__ void stage_fixed(const C2<T>* __restrict__ in, C2<T>* __restrict__ out,
                                            const C2<T>* __restrict__ tw, int n, int Ns, int nlc) {
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  for (int u = threadIdx.x; u < nlc * nb; u += blockDim.x) {
    const int line = u / nb;
    const int jj = u - line * nb;
    const C2<T>* li = in + line * n;
    C2<T>* lo = out + line * n;
    const int kk = jj % Ns;
    C2<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = li[jj + r * nb];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * kk * twstep]);
    }
    if (R == 2) dft2(v);
    if (R == 4) dft4(v);
    if (R == 8) dft8(v);
    const int base = (jj / Ns) * Ns * R + kk;
#pragma unroll
    for (int r = 0; r < R; ++r) lo[base + r * Ns] = v[r];
  }
}

// one Stockham stage with any radix R (direct DFT, used for odd factors)
template <typename T>
__device__ __forceinline__ void stage_generic(const C2<T>* __restrict__ in, C2<T>* __restrict__ out,
                                              const C2<T>* __restrict__ tw, int n, int Ns, int R,
                                              int nlc) {
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  const int wstep = n / R;
  for (int u = threadIdx.x; u < nlc * nb; u += blockDim.x) {
    const int line = u / nb;
    const int jj = u - line * nb;
    const C2<T>* li = in + line * n;
    C2<T>* lo = out + line * n;
    const int kk = jj % Ns;
    const int base = (jj / Ns) * Ns * R + kk;
    for (int p = 0; p < R; ++p) {
      C2<T> acc = {T(0), T(0)};
      for (int r = 0; r < R; ++r) {
        C2<T> x = li[jj + r * nb];
        if (Ns > 1 && r > 0) x = cmul(x, tw[r * kk * twstep]);
        acc = cadd(acc, cmul(x, tw[((p * r) % R) * wstep]));
      }
      lo[base + p * Ns] = acc;
    }
  }
}

// full complex FFT of nlc lines held in LDS; returns the buffer holding the result
template <typename T>
__device__ C2<T>* fft_lines(C2<T>* bufA, C2<T>* bufB, const C2<T>* __restrict__ tw,
                            const DhtArgs& A, int nlc) {
  C2<T>* in = bufA;
  C2<T>* out = bufB;
  int Ns = 1;
  for (int s = 0; s < A.nstages; ++s) {
    const int R = A.radix[s];
    if (R == 8)
      stage_fixed<T, 8>(in, out, tw, A.n, Ns, nlc);
    else if (R == 4)
      stage_fixed<T, 4>(in, out, tw, A.n, Ns, nlc);
    else if (R == 2)
      stage_fixed<T, 2>(in, out, tw, A.n, Ns, nlc);
    else
      stage_generic<T>(in, out, tw, A.n, Ns, R, nlc);
    __syncthreads();
    C2<T>* t = in;
    in = out;
    out = t;
    Ns *= R;
  }
  return in;
}

// tile element e -> (sample s, line t); the fastest index is the unit-stride one
template <bool CONTIG>
__device__ __forceinline__ void tile_coords(int e, int n, int nl, int& s, int& t) {
  if (CONTIG) {
    t = e / n;
    s = e - t * n;
  } else {
    s = e / nl;
    t = e - s * nl;
  }
}

template <typename T>
__device__ __forceinline__ T hartley_of(const C2<T>* F, int n, int t, int s) {
  const C2<T> zq = F[(t >> 1) * n + s];
  const C2<T> zm = F[(t >> 1) * n + (s == 0 ? 0 : n - s)];
  if ((t & 1) == 0) return T(0.5) * ((zq.x + zm.x) - (zq.y - zm.y));
  return T(0.5) * ((zq.y + zm.y) + (zq.x - zm.x));
}

// One Hartley pass over a tile; MIDDLE additionally applies m(q) and the second
// transform along the same axis (the axis-1 pass of the solve).
template <typename T, bool CONTIG, bool MIDDLE>
__global__ void __launch_bounds__(kThreads)
k_hartley(T* __restrict__ data, const C2<T>* __restrict__ tw, DhtArgs A,
          const T* __restrict__ s1, const T* __restrict__ s2, const T* __restrict__ s3,
          const Prob* __restrict__ prob) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.y;
  if (prob != nullptr && prob[b].done) return;
  const int n = A.n, nl = A.nl, nlc = nl >> 1;
  C2<T>* bufA = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* bufB = bufA + nlc * n;
  T* bufAr = reinterpret_cast<T*>(bufA);

  const int outer = blockIdx.x / A.tiles_per_outer;
  const int lt = blockIdx.x - outer * A.tiles_per_outer;
  const int line0 = lt * nl;
  const int nvalid = min(nl, A.lines_total - line0);
  T* base = data + (size_t)b * A.field_stride + (size_t)outer * A.os + (size_t)line0 * A.ls;

  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int s, t;
    tile_coords<CONTIG>(e, n, nl, s, t);
    const T v = (t < nvalid) ? base[(size_t)s * A.ss + (size_t)t * A.ls] : T(0);
    bufAr[((t >> 1) * n + s) * 2 + (t & 1)] = v;
  }
  __syncthreads();
  C2<T>* F = fft_lines<T>(bufA, bufB, tw, A, nlc);

  if (MIDDLE) {
    // H along axis 0 is known; scale by m(q1, q2, q3) and transform again
    C2<T>* G = (F == bufA) ? bufB : bufA;
    T* Gr = reinterpret_cast<T*>(G);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
      int s, t;
      tile_coords<CONTIG>(e, n, nl, s, t);
      const int q2 = outer, q3 = line0 + t;
      T h = hartley_of<T>(F, n, t, s);
      T m = T(0);
      if (t < nvalid) {
        const T lam = s1[s] + s2[q2] + s3[q3];
        m = (lam > T(0)) ? T(A.scale) / lam : T(0);  // lambda = -lam; sign applied below
      }
      Gr[((t >> 1) * n + s) * 2 + (t & 1)] = -h * m;
    }
    __syncthreads();
    // fft_lines ping-pongs between its two arguments starting from the first
    F = fft_lines<T>(G, (G == bufA) ? bufB : bufA, tw, A, nlc);
  }

  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int s, t;
    tile_coords<CONTIG>(e, n, nl, s, t);
    if (t < nvalid) base[(size_t)s * A.ss + (size_t)t * A.ls] = hartley_of<T>(F, n, t, s);
  }
}

}  // namespace ccmf
