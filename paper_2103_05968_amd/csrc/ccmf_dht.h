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

#include <type_traits>

#include "ccmf_fft_pow2.h"
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
  int32_t lognl;        // log2(nl) for the power-of-two kernel
  int32_t vec;          // power-of-two kernel: vector loads/stores are aligned
  int32_t outers;       // power-of-two kernel: number of outer indices
  int32_t walk;         // power-of-two kernel: tiles walked per block
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
// transform along the same axis (the axis-1 pass of the solve).  Samples are
// loaded as TI, transformed in TC (LDS and twiddles) and stored as TO, so the
// half of the solve after the division by lambda can run in FP64 for FP32
// fields: the potential has magnitude O(N) while the update needs its O(1)
// differences.  `in` and `out` have the same layout and may alias.
template <typename TI, typename TO, typename TC, bool CONTIG, bool MIDDLE>
__global__ void __launch_bounds__(kThreads)
k_hartley(const TI* in, TO* out, const C2<TC>* __restrict__ tw, DhtArgs A,
          const TC* __restrict__ s1, const TC* __restrict__ s2, const TC* __restrict__ s3,
          const Prob* __restrict__ prob) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.y;
  if (prob != nullptr && prob[b].done) return;
  const int n = A.n, nl = A.nl, nlc = nl >> 1;
  C2<TC>* bufA = reinterpret_cast<C2<TC>*>(smem_raw);
  C2<TC>* bufB = bufA + nlc * n;
  TC* bufAr = reinterpret_cast<TC*>(bufA);

  const int outer = blockIdx.x / A.tiles_per_outer;
  const int lt = blockIdx.x - outer * A.tiles_per_outer;
  const int line0 = lt * nl;
  const int nvalid = min(nl, A.lines_total - line0);
  const size_t off = (size_t)b * A.field_stride + (size_t)outer * A.os + (size_t)line0 * A.ls;
  const TI* src = in + off;
  TO* dst = out + off;

  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int s, t;
    tile_coords<CONTIG>(e, n, nl, s, t);
    const TC v = (t < nvalid) ? TC(src[(size_t)s * A.ss + (size_t)t * A.ls]) : TC(0);
    bufAr[((t >> 1) * n + s) * 2 + (t & 1)] = v;
  }
  __syncthreads();
  C2<TC>* F = fft_lines<TC>(bufA, bufB, tw, A, nlc);

  if (MIDDLE) {
    // H along axis 0 is known; scale by m(q1, q2, q3) = 1/(lambda N) and transform again
    C2<TC>* G = (F == bufA) ? bufB : bufA;
    TC* Gr = reinterpret_cast<TC*>(G);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
      int s, t;
      tile_coords<CONTIG>(e, n, nl, s, t);
      const int q2 = outer, q3 = line0 + t;
      const TC h = hartley_of<TC>(F, n, t, s);
      TC m = TC(0);
      if (t < nvalid) {
        const TC lam = s1[s] + s2[q2] + s3[q3];   // lambda(q) = -lam
        m = (lam > TC(0)) ? -TC(A.scale) / lam : TC(0);
      }
      Gr[((t >> 1) * n + s) * 2 + (t & 1)] = h * m;
    }
    __syncthreads();
    F = fft_lines<TC>(G, (G == bufA) ? bufB : bufA, tw, A, nlc);
  }

  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int s, t;
    tile_coords<CONTIG>(e, n, nl, s, t);
    if (t < nvalid) dst[(size_t)s * A.ss + (size_t)t * A.ls] = TO(hartley_of<TC>(F, n, t, s));
  }
}


// ---------------------------------------------------------------------------
// Power-of-two line lengths: compile-time plan (ccmf_fft_pow2.h).  The block
// holds NLC = blockDim / TPL complex lines (2 NLC real lines), each padded by one
// element so that the line-strided LDS accesses of the column passes spread
// over the banks.  Stages run in place: read E values, compute, barrier, write.
// ---------------------------------------------------------------------------
// LDS position of line element p: one padding slot every E elements, so the
// stride-E accesses of a stage (thread t writing t*E + r) spread over the banks.
template <int N, int V>
__device__ __forceinline__ int pidx(int p) {
  return p + p / pow2::Plan<N, V>::E;
}
template <int N, int V>
constexpr int line_pitch() {
  return N + N / pow2::Plan<N, V>::E + 1;  // odd pitch: consecutive lines start on different banks
}

template <typename TC, int N, int V>
__device__ __forceinline__ void fft_line_p2(pow2::CX<TC>* line, int t, const pow2::CX<TC>* __restrict__ tw) {
  using P = pow2::Plan<N, V>;
  constexpr int E = P::E, TPL = N / E;
  pow2::CX<TC> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = line[pidx<N, V>(t + TPL * e)];
  pow2::stage_compute<TC, N, E, P::R0, 1>(v, t, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E / P::R0; ++m)
#pragma unroll
    for (int r = 0; r < P::R0; ++r)
      line[pidx<N, V>(pow2::stage_out_pos<N, E, P::R0, 1>(t, m, r))] = v[m + r * (E / P::R0)];
  __syncthreads();
  if constexpr (P::R1 > 0) {
    constexpr int NS = P::R0;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = line[pidx<N, V>(t + TPL * e)];
    pow2::stage_compute<TC, N, E, P::R1, NS>(v, t, tw);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / P::R1; ++m)
#pragma unroll
      for (int r = 0; r < P::R1; ++r)
        line[pidx<N, V>(pow2::stage_out_pos<N, E, P::R1, NS>(t, m, r))] = v[m + r * (E / P::R1)];
    __syncthreads();
  }
  if constexpr (P::R2 > 0) {
    constexpr int NS = P::R0 * P::R1;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = line[pidx<N, V>(t + TPL * e)];
    pow2::stage_compute<TC, N, E, P::R2, NS>(v, t, tw);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / P::R2; ++m)
#pragma unroll
      for (int r = 0; r < P::R2; ++r)
        line[pidx<N, V>(pow2::stage_out_pos<N, E, P::R2, NS>(t, m, r))] = v[m + r * (E / P::R2)];
    __syncthreads();
  }
  if constexpr (P::R3 > 0) {
    constexpr int NS = P::R0 * P::R1 * P::R2;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = line[pidx<N, V>(t + TPL * e)];
    pow2::stage_compute<TC, N, E, P::R3, NS>(v, t, tw);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / P::R3; ++m)
#pragma unroll
      for (int r = 0; r < P::R3; ++r)
        line[pidx<N, V>(pow2::stage_out_pos<N, E, P::R3, NS>(t, m, r))] = v[m + r * (E / P::R3)];
    __syncthreads();
  }
}

template <typename TC, int N, int V>
__device__ __forceinline__ TC hartley_p2(const pow2::CX<TC>* L, int lp, int line, int s) {
  const pow2::CX<TC> zq = L[(line >> 1) * lp + pidx<N, V>(s)];
  const pow2::CX<TC> zm = L[(line >> 1) * lp + pidx<N, V>((N - s) & (N - 1))];
  if ((line & 1) == 0) return TC(0.5) * ((zq.x + zm.x) - (zq.y - zm.y));
  return TC(0.5) * ((zq.y + zm.y) + (zq.x - zm.x));
}

template <bool CONTIG, int N>
__device__ __forceinline__ void tile_coords_p2(int e, int lognl, int& s, int& line) {
  if (CONTIG) {
    line = e / N;
    s = e & (N - 1);
  } else {
    s = e >> lognl;
    line = e & ((1 << lognl) - 1);
  }
}

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// Input samples of one tile held in registers between the global loads and the
// LDS tile, so that the loads of the next tile are in flight while the current
// tile is transformed.  Rows (CONTIG): IT iterations of two VW-vectors (the two
// rows of a pair); columns: IT iterations of one 2-vector (both lines of a pair
// are adjacent in memory).
template <typename TI, int N, int E, bool CONTIG>
struct TileRegs {
  static constexpr int VW = CONTIG ? 16 / (int)sizeof(TI) : 2;
  static constexpr int TPL = N / E;
  static constexpr int CH = N >= VW ? N / VW : 1;
  static constexpr int IT = CONTIG ? (CH + TPL - 1) / TPL : E;
  VecT<TI, VW> va[IT];
  VecT<TI, VW> vb[CONTIG ? IT : 1];
};

// One Hartley pass over a tile of `nl` lines; MIDDLE additionally scales by
// m(q) and transforms again along the same axis (see k_hartley).  A block walks
// A.walk tiles at a stride of the grid size (so the blocks running together
// always work on adjacent tiles, which share the 128-byte lines of a row in
// L2), loading the next tile's samples into registers before it transforms the
// current one.
// With FP32 samples and FP64 compute (the middle pass of FP32 fields) the
// forward transform runs in FP32 like the other forward passes (tw32: its
// twiddles) and the coefficients are widened to FP64 before the scaling, so
// the inverse transform and the potential are FP64.
template <typename TI, typename TO, typename TC, int N, int V, bool CONTIG, bool MIDDLE>
__global__ void __launch_bounds__(512)
k_hartley_p2(const TI* in, TO* out, const pow2::CX<TC>* __restrict__ tw, const pow2::CX<float>* __restrict__ tw32,
             DhtArgs A, const TC* __restrict__ s1, const TC* __restrict__ s2, const TC* __restrict__ s3,
             const Prob* __restrict__ prob) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.y;
  if (prob != nullptr && prob[b].done) return;
  using P = pow2::Plan<N, V>;
  constexpr int E = P::E, TPL = N / E, LP = line_pitch<N, V>();
  using RG = TileRegs<TI, N, E, CONTIG>;
  constexpr bool F32FWD = MIDDLE && sizeof(TI) == 4 && sizeof(TC) == 8;
  using TF = typename std::conditional<F32FWD, float, TC>::type;  // forward transform type
  const int nl = 1 << A.lognl;
  pow2::CX<TC>* L = reinterpret_cast<pow2::CX<TC>*>(smem_raw);
  pow2::CX<TF>* LF = reinterpret_cast<pow2::CX<TF>*>(smem_raw);  // same tile, forward type
  TF* LFr = reinterpret_cast<TF*>(smem_raw);
  const int c = threadIdx.x / TPL, t = threadIdx.x & (TPL - 1);
  const int total = nl * N;
  const TI* src_b = in + (size_t)b * A.field_stride;
  TO* dst_b = out + (size_t)b * A.field_stride;

  // twiddle table of this length staged in LDS behind the data tile (and the
  // FP32 table of the forward transform behind it)
  pow2::CX<TC>* twl = L + (size_t)(nl >> 1) * LP;
  for (int j = threadIdx.x; j < N; j += blockDim.x) twl[j] = tw[j];
  pow2::CX<TF>* twf = reinterpret_cast<pow2::CX<TF>*>(twl);
  if constexpr (F32FWD) {
    twf = reinterpret_cast<pow2::CX<TF>*>(twl + N);
    for (int j = threadIdx.x; j < N; j += blockDim.x) twf[j] = tw32[j];
  }

  // XCD-contiguous tiles: neighbouring tiles share the 128-byte lines of a row
  const int ntiles = A.outers * A.tiles_per_outer;
  const int tile0 = xcd_remap(blockIdx.x, gridDim.x);
  const int tstride = (int)gridDim.x;  // gridDim.x * A.walk >= ntiles
  const int tile_end = min(tile0 + A.walk * tstride, ntiles);

  auto tile_base = [&](int tile, int& outer, int& line0, int& nvalid) -> size_t {
    outer = tile / A.tiles_per_outer;
    line0 = (tile - outer * A.tiles_per_outer) * nl;
    nvalid = min(nl, A.lines_total - line0);
    return (size_t)outer * A.os + (size_t)line0 * A.ls;
  };
  // global -> registers (vector paths)
  auto load_regs = [&](int tile, RG& R) {
    int outer, line0, nvalid;
    const TI* src = src_b + tile_base(tile, outer, line0, nvalid);
#pragma unroll
    for (int it = 0; it < RG::IT; ++it) {
      const int e = threadIdx.x + it * (int)blockDim.x;
      if constexpr (CONTIG) {
        // e < (nl/2) CH except for plans with fewer than VW samples per thread
        if (RG::IT * TPL == RG::CH || e < (nl >> 1) * RG::CH) {
          const int pr = e / RG::CH, s0 = (e & (RG::CH - 1)) * RG::VW;
          const int ra = min(2 * pr, nvalid - 1), rb = min(2 * pr + 1, nvalid - 1);
          R.va[it] = *reinterpret_cast<const VecT<TI, RG::VW>*>(src + (size_t)ra * A.ls + s0);
          R.vb[it] = *reinterpret_cast<const VecT<TI, RG::VW>*>(src + (size_t)rb * A.ls + s0);
        }
      } else {
        // pairs are whole: n3 and nl are even, so nvalid is even
        const int lognlc = A.lognl - 1;
        const int sp = e >> lognlc, pr = min(e & ((1 << lognlc) - 1), (nvalid >> 1) - 1);
        R.va[it] = *reinterpret_cast<const VecT<TI, 2>*>(src + (size_t)sp * A.ss + 2 * pr);
      }
    }
  };
  // registers -> LDS tile
  auto put_regs = [&](const RG& R, int nvalid) {
#pragma unroll
    for (int it = 0; it < RG::IT; ++it) {
      const int e = threadIdx.x + it * (int)blockDim.x;
      if constexpr (CONTIG) {
        if (RG::IT * TPL == RG::CH || e < (nl >> 1) * RG::CH) {
          const int pr = e / RG::CH, s0 = (e & (RG::CH - 1)) * RG::VW;
          const bool oka = 2 * pr < nvalid, okb = 2 * pr + 1 < nvalid;
#pragma unroll
          for (int v = 0; v < RG::VW; ++v)
            LF[pr * LP + pidx<N, V>(s0 + v)] = {oka ? TF(R.va[it].v[v]) : TF(0), okb ? TF(R.vb[it].v[v]) : TF(0)};
        }
      } else {
        const int lognlc = A.lognl - 1;
        const int sp = e >> lognlc, pr = e & ((1 << lognlc) - 1);
        const bool ok = 2 * pr < nvalid;
        LF[pr * LP + pidx<N, V>(sp)] = {ok ? TF(R.va[it].v[0]) : TF(0), ok ? TF(R.va[it].v[1]) : TF(0)};
      }
    }
  };

  RG R;
  if (A.vec && tile0 < tile_end) load_regs(tile0, R);
  for (int tile = tile0; tile < tile_end; tile += tstride) {
    int outer, line0, nvalid;
    const size_t off = tile_base(tile, outer, line0, nvalid);
    if (A.vec) {
      put_regs(R, nvalid);
    } else {
      const TI* src = src_b + off;
      for (int e = threadIdx.x; e < total; e += blockDim.x) {
        int s, l;
        tile_coords_p2<CONTIG, N>(e, A.lognl, s, l);
        const TF v = (l < nvalid) ? TF(src[(size_t)s * A.ss + (size_t)l * A.ls]) : TF(0);
        LFr[((l >> 1) * LP + pidx<N, V>(s)) * 2 + (l & 1)] = v;
      }
    }
    __syncthreads();
    // the next tile's loads overlap this tile's transforms
    if (A.vec && tile + tstride < tile_end) load_regs(tile + tstride, R);
    fft_line_p2<TF, N, V>(LF + c * LP, t, twf);

    if constexpr (MIDDLE) {
      // Scale the Hartley coefficients by m(q) = 1/(lambda(q) N) and repack them
      // as the next transform's input.  Positions s and N-s of a complex line hold
      // both coefficients of its two real lines at s and N-s, and lambda(s) =
      // lambda(N-s), so each thread rewrites its own pairs.
      const int la = 2 * c, lb = 2 * c + 1;
      const TC sa = (la < nvalid) ? s2[outer] + s3[line0 + la] : TC(-1);
      const TC sb = (lb < nvalid) ? s2[outer] + s3[line0 + lb] : TC(-1);
      pow2::CX<TC>* Lc = L + c * LP;
      auto scale_pair = [&](int sp, const pow2::CX<TC>& zs, const pow2::CX<TC>& zm) {
        const int sm = (N - sp) & (N - 1);
        const TC ha_s = TC(0.5) * ((zs.x + zm.x) - (zs.y - zm.y));
        const TC hb_s = TC(0.5) * ((zs.y + zm.y) + (zs.x - zm.x));
        const TC ha_m = TC(0.5) * ((zm.x + zs.x) - (zm.y - zs.y));
        const TC hb_m = TC(0.5) * ((zm.y + zs.y) + (zm.x - zs.x));
        const TC s1v = s1[sp];
        const TC lam_a = s1v + sa, lam_b = s1v + sb;     // lambda(q) = -lam
        const TC ma = (sa >= TC(0) && lam_a > TC(0)) ? -TC(A.scale) / lam_a : TC(0);
        const TC mb = (sb >= TC(0) && lam_b > TC(0)) ? -TC(A.scale) / lam_b : TC(0);
        Lc[pidx<N, V>(sp)] = {ha_s * ma, hb_s * mb};
        Lc[pidx<N, V>(sm)] = {ha_m * ma, hb_m * mb};
      };
      if constexpr (F32FWD) {
        // the FP64 tile overlays the FP32 one: the FP32 pairs of this thread
        // (s = t + TPL q <= N/2) are read before the barrier, written after it
        constexpr int NP = N / 2 / TPL + 1;
        const pow2::CX<TF>* LFc = LF + c * LP;
        pow2::CX<TF> fs[NP], fm[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int sp = t + q * TPL;
          if (sp <= N / 2) {
            fs[q] = LFc[pidx<N, V>(sp)];
            fm[q] = LFc[pidx<N, V>((N - sp) & (N - 1))];
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int sp = t + q * TPL;
          if (sp <= N / 2) scale_pair(sp, {TC(fs[q].x), TC(fs[q].y)}, {TC(fm[q].x), TC(fm[q].y)});
        }
      } else {
        for (int sp = t; sp <= N / 2; sp += TPL) {
          const pow2::CX<TC> zs = Lc[pidx<N, V>(sp)], zm = Lc[pidx<N, V>((N - sp) & (N - 1))];
          scale_pair(sp, zs, zm);
        }
      }
      __syncthreads();
      fft_line_p2<TC, N, V>(L + c * LP, t, twl);
    }

    TO* dst = dst_b + off;
    if (A.vec) {
      if constexpr (CONTIG) {
        constexpr int VW = 16 / sizeof(TO);
        constexpr int CH = N >= VW ? N / VW : 1;
        for (int e = threadIdx.x; e < (nl >> 1) * CH; e += blockDim.x) {
          const int pr = e / CH, s0 = (e & (CH - 1)) * VW;
          VecT<TO, VW> va, vb;
#pragma unroll
          for (int v = 0; v < VW; ++v) {
            va.v[v] = TO(hartley_p2<TC, N, V>(L, LP, 2 * pr, s0 + v));
            vb.v[v] = TO(hartley_p2<TC, N, V>(L, LP, 2 * pr + 1, s0 + v));
          }
          if (2 * pr < nvalid) *reinterpret_cast<VecT<TO, VW>*>(dst + (size_t)(2 * pr) * A.ls + s0) = va;
          if (2 * pr + 1 < nvalid) *reinterpret_cast<VecT<TO, VW>*>(dst + (size_t)(2 * pr + 1) * A.ls + s0) = vb;
        }
      } else {
        const int lognlc = A.lognl - 1;
        for (int e = threadIdx.x; e < (nl >> 1) * N; e += blockDim.x) {
          const int sp = e >> lognlc, pr = e & ((1 << lognlc) - 1);
          if (2 * pr < nvalid) {
            VecT<TO, 2> v2;
            v2.v[0] = TO(hartley_p2<TC, N, V>(L, LP, 2 * pr, sp));
            v2.v[1] = TO(hartley_p2<TC, N, V>(L, LP, 2 * pr + 1, sp));
            *reinterpret_cast<VecT<TO, 2>*>(dst + (size_t)sp * A.ss + 2 * pr) = v2;
          }
        }
      }
    } else {
      for (int e = threadIdx.x; e < total; e += blockDim.x) {
        int s, l;
        tile_coords_p2<CONTIG, N>(e, A.lognl, s, l);
        if (l < nvalid) dst[(size_t)s * A.ss + (size_t)l * A.ls] = TO(hartley_p2<TC, N, V>(L, LP, l, s));
      }
    }
    // the tile is rewritten by the next iteration
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// r = div^- A* w (the argument of the spectral solve, eq:CCMF_FFT_Gamma_2) fused
// with the forward Hartley pass along k: a block forms r for nl whole k-rows of
// one plane straight into its LDS tile, transforms them and writes the k-Hartley
// coefficients, so r itself never goes through HBM.  Rows of a block are
// consecutive j at fixed i; a block walks `planes` consecutive planes.  N = n3.
// ---------------------------------------------------------------------------
struct DivArgs {
  int32_t n1, n2, n3;
  int32_t nl, lognl;       // real lines (rows) per tile
  int32_t jtiles;          // ceil(n2 / nl)
  int32_t planes;          // planes walked per block
  int32_t ichunks;         // ceil(n1 / planes)
  int32_t vec;             // vector stores allowed
};

template <typename T, int N, int V>
__global__ void __launch_bounds__(512)
k_div_hartley_p2(const T* __restrict__ z, const T* __restrict__ a, T* __restrict__ rout,
                 const pow2::CX<T>* __restrict__ tw, DivArgs D, const Prob* __restrict__ prob) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  if (P.done) return;
  using PL = pow2::Plan<N, V>;
  constexpr int E = PL::E, TPL = N / E, LP = line_pitch<N, V>();
  const int nl = D.nl;
  pow2::CX<T>* L = reinterpret_cast<pow2::CX<T>*>(smem_raw);
  T* Lr = reinterpret_cast<T*>(smem_raw);
  pow2::CX<T>* twl = L + (size_t)(nl >> 1) * LP;
  for (int j = threadIdx.x; j < N; j += blockDim.x) twl[j] = tw[j];
  const int c = threadIdx.x / TPL, t = threadIdx.x & (TPL - 1);

  const T ir = T(1.0 / P.rho), irp = T(1.0 / P.rho_prev);
  const uint32_t n23 = (uint32_t)D.n2 * N, NN = (uint32_t)D.n1 * n23;
  const T* zb = z + (size_t)b * 6 * NN;
  const T* ab = a + (size_t)b * NN;
  T* rb = rout + (size_t)b * NN;

  const int bx = xcd_remap(blockIdx.x, gridDim.x);
  const int jt = bx % D.jtiles, ic = bx / D.jtiles;
  const int j0 = jt * nl;
  const int nvalid = min(nl, D.n2 - j0);
  for (int step = 0; step < D.planes; ++step) {
    const int i = ic * D.planes + step;
    if (i >= D.n1) break;
    const uint32_t ip = (i + 1 == D.n1) ? 0u : (uint32_t)(i + 1);
    const uint32_t im = (i == 0) ? (uint32_t)(D.n1 - 1) : (uint32_t)(i - 1);
    // r for the tile's rows, written into the LDS tile as real lines.  The loop
    // has 2E trips (blockDim = nl N / (2E)); the samples of U elements are loaded
    // first, branch-free (rows past the edge of the cell read row n2 - 1 and are
    // zeroed afterwards), so that their loads are in flight together.
    constexpr int ITS = 2 * E;
    constexpr int U = sizeof(T) == 8 ? 2 : 4;
    static_assert(ITS % U == 0, "trip count");
    for (int g0 = 0; g0 < ITS; g0 += U) {
      T zc[U][6], ac[U], ap[U][3], zp[U][3], am[U][3], zm[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = threadIdx.x + (g0 + u) * (int)blockDim.x;
        const int l = e / N, k = e & (N - 1);
        const uint32_t j = (uint32_t)min(j0 + l, D.n2 - 1);
        const uint32_t jp = (j + 1 == (uint32_t)D.n2) ? 0u : j + 1;
        const uint32_t jm = (j == 0) ? (uint32_t)(D.n2 - 1) : j - 1;
        const uint32_t kp = (k + 1 == N) ? 0u : (uint32_t)(k + 1);
        const uint32_t km = (k == 0) ? (uint32_t)(N - 1) : (uint32_t)(k - 1);
        const uint32_t row = (uint32_t)i * n23 + j * N;
        const uint32_t x = row + k;
        const uint32_t xp[3] = {ip * n23 + j * N + k, (uint32_t)i * n23 + jp * N + k, row + kp};
        const uint32_t xm[3] = {im * n23 + j * N + k, (uint32_t)i * n23 + jm * N + k, row + km};
        ac[u] = ab[x];
#pragma unroll
        for (int q = 0; q < 6; ++q) zc[u][q] = zb[(size_t)q * NN + x];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          ap[u][q] = ab[xp[q]];
          zp[u][q] = zb[(size_t)(q + 3) * NN + xp[q]];
          am[u][q] = ab[xm[q]];
          zm[u][q] = zb[(size_t)q * NN + xm[q]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = threadIdx.x + (g0 + u) * (int)blockDim.x;
        const int l = e / N, k = e & (N - 1);
        const T bx0 = beta_of(ac[u], irp, ir);
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const T w1 = bx0 * zc[u][q];
          const T w2 = bx0 * zc[u][q + 3];
          const T w2p = beta_of(ap[u][q], irp, ir) * zp[u][q];
          const T w1m = beta_of(am[u][q], irp, ir) * zm[u][q];
          acc += (w1 + w2p) - (w1m + w2);
        }
        const T rv = (l < nvalid) ? acc * T(0.70710678118654752440) : T(0);
        Lr[((l >> 1) * LP + pidx<N, V>(k)) * 2 + (l & 1)] = rv;
      }
    }
    __syncthreads();
    fft_line_p2<T, N, V>(L + c * LP, t, twl);
    // k-Hartley coefficients of the tile's rows
    T* dst = rb + (size_t)i * n23 + (size_t)j0 * N;
    if (D.vec) {
      constexpr int VW = 16 / sizeof(T);
      constexpr int CH = N >= VW ? N / VW : 1;  // vector stores only for N * sizeof(T) >= 16
      for (int e = threadIdx.x; e < (nl >> 1) * CH; e += blockDim.x) {
        const int pr = e / CH, s0 = (e & (CH - 1)) * VW;
        VecT<T, VW> va, vb;
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          va.v[v] = hartley_p2<T, N, V>(L, LP, 2 * pr, s0 + v);
          vb.v[v] = hartley_p2<T, N, V>(L, LP, 2 * pr + 1, s0 + v);
        }
        if (2 * pr < nvalid) *reinterpret_cast<VecT<T, VW>*>(dst + (size_t)(2 * pr) * N + s0) = va;
        if (2 * pr + 1 < nvalid) *reinterpret_cast<VecT<T, VW>*>(dst + (size_t)(2 * pr + 1) * N + s0) = vb;
      }
    } else {
      for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
        const int l = e / N, k = e & (N - 1);
        if (l < nvalid) dst[(size_t)l * N + k] = hartley_p2<T, N, V>(L, LP, l, k);
      }
    }
    __syncthreads();
  }
}

}  // namespace ccmf
