// Device kernels of the CCMF ADMM (Ernesti & Schneider, arXiv 2103.05968, Sec. 3).
//
// State representation.  The paper iterates the pair (v^k, e^k) of 6-component
// fields.  The e/v update of eq:CCMF_FFT_ADMM writes both from one 6-vector
// z = v^k + rho^k xi^{k+1}:  v^{k+1} = P_C(z) = alpha z with
// alpha = min(1, gamma/|z|), and e^{k+1} = (1 - alpha) z / rho^k.  The kernels
// therefore keep z (6 reals) and alpha (1 real) per voxel instead of (v, e)
// (12 reals) and rebuild v, e and w = e - v/rho on the fly:
//     w = beta z,   beta = (1 - alpha)/rho^{k-1} - alpha/rho^k.
// Both pairs are ping-ponged (the update reads neighbours of the old state).
//
// Geometry.  C-order [N1][N2][N3], k fastest; field b occupies [b*N, (b+1)*N).
// Shifts are periodic: x +- e_c wraps inside the cell (Sec. 2.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmf {

constexpr int kThreads = 256;
// threads per block (= voxels per tile) of the stencil kernels k_div and k_update
constexpr int kUpd = 256;
// blocks per problem of the stencil kernels (each walks tiles, see tile_of) and
// FP64 partial rows per problem.  Measured on MI355X (256^3, FP32): fewer tiles
// per block make k_update faster by a few percent (4 planes: -4 %), but the
// extra reduction level that the larger number of partial rows needs costs more
// than that (one more launch per iteration).
constexpr int kUpdBlocks = 2048;
constexpr int kNQ = 16;  // FP64 partial sums per block (13 used)

// indices of the per-block FP64 partial sums
enum {
  Q_RES2 = 0,  // sum |e^k - xi^{k+1/2}|^2
  Q_MV = 1,    // 6 sums of v^k components (mean multiplier)
  Q_E = 7,     // sum gamma |xi^{k+1/2}|   (primal energy)
  Q_BBN = 8,   // sum <v^{k+1} - v^k, e^{k+1} - e^k>
  Q_BBD = 9,   // sum |e^{k+1} - e^k|^2
  Q_VV = 10,   // sum |v^{k+1}|^2
  Q_EE = 11,   // sum |e^{k+1}|^2
  Q_DUAL = 12,  // sum <A xibar, v^k>
  Q_DVV = 13    // sum |v^{k+1} - v^k|^2
};
constexpr int kNQU = 14;  // partial sums in use

// Per-problem scalars, device resident.  Written by the host before the first
// iteration, afterwards only by k_finish (one thread).
struct Prob {
  double rho;       // rho^k, penalty of the running iteration
  double rho_prev;  // rho^{k-1}: e^k = (1 - alpha) z / rho_prev
  double rho0, lo, hi, tol, delta;
  double bb_corr, eta0, k0;
  double xibar[3];
  double geff, res, mvn, dual;
  double mflux[3];  // mean face flux <A* v^k> at the stopping iterate
  int32_t k;        // iteration index of the current state within this solve
  int32_t k_off;    // iterations before this solve (warm start); the global index is k_off + k
  int32_t done;     // 0 running, 1 converged, 2 stopped at max_iter
  int32_t rule, max_iter, all_zero, field;
};

struct Geo {
  int32_t n1, n2, n3, n23;
  uint32_t N;
  int32_t nloads;
  int32_t tiles;        // ceil(N / kUpd)
  int32_t tiles_per_blk;
  int32_t tpp;          // tiles per i-plane when n2*n3 % kUpd == 0, else 0
};

// Tile visited by logical block lb at step m.  With whole tiles per plane, a
// block walks tiles_per_blk consecutive planes at one in-plane tile, so the
// i-1 and i+1 rows it reads are its own previous and next steps; adjacent
// logical blocks take adjacent in-plane tiles (the j neighbours).  Otherwise
// a block takes tiles_per_blk consecutive tiles.
__device__ __forceinline__ int tile_of(const Geo& g, int lb, int m) {
  if (g.tpp > 0) {
    const int u = lb % g.tpp, c = lb / g.tpp;
    return (c * g.tiles_per_blk + m) * g.tpp + u;
  }
  return lb * g.tiles_per_blk + m;
}

__device__ __forceinline__ int xcd_remap(int w, int G) {
  // Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; give
  // each XCD a contiguous slab of logical tiles so stencil neighbours share its L2.
  const int G8 = G & ~7;
  if (w >= G8) return w;
  const int per = G8 >> 3;
  return (w & 7) * per + (w >> 3);
}

struct Nbr {
  uint32_t p[3], m[3];  // linear index of x + e_c and x - e_c
};

__device__ __forceinline__ Nbr neighbours(const Geo& g, uint32_t x) {
  const uint32_t i = x / (uint32_t)g.n23;
  const uint32_t rem = x - i * (uint32_t)g.n23;
  const uint32_t j = rem / (uint32_t)g.n3;
  const uint32_t k = rem - j * (uint32_t)g.n3;
  Nbr nb;
  const uint32_t s0 = g.n23, s1 = g.n3;
  nb.p[0] = (i + 1 == (uint32_t)g.n1) ? x - i * s0 : x + s0;
  nb.m[0] = (i == 0) ? x + (uint32_t)(g.n1 - 1) * s0 : x - s0;
  nb.p[1] = (j + 1 == (uint32_t)g.n2) ? x - j * s1 : x + s1;
  nb.m[1] = (j == 0) ? x + (uint32_t)(g.n2 - 1) * s1 : x - s1;
  nb.p[2] = (k + 1 == (uint32_t)g.n3) ? x - k : x + 1;
  nb.m[2] = (k == 0) ? x + (uint32_t)(g.n3 - 1) : x - 1;
  return nb;
}

template <typename T>
__device__ __forceinline__ T beta_of(T alpha, T inv_rho_prev, T inv_rho) {
  return (T(1) - alpha) * inv_rho_prev - alpha * inv_rho;
}

template <typename T>
__device__ __forceinline__ T ball_scale(T nz, T gam) {
  // P_C(z) = alpha z (eq:CCMF_FFT_Cgamma): alpha = gamma/|z| outside the ball, else 1
  return nz > gam ? gam / nz : T(1);
}

// ---------------------------------------------------------------------------
// Initial state (planar crack, v^0 in the subdifferential of g at e^0):
// e^0 = A xibar, v^0 = gamma A xibar, stored as z^0 = (gamma + rho0) A xibar.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_init(Geo g, const T* __restrict__ kap, T* __restrict__ z, T* __restrict__ a,
       const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  const T* gam = kap + (size_t)P.field * g.N;
  T* zb = z + (size_t)b * 6 * g.N;
  T* ab = a + (size_t)b * g.N;
  const T s = T(0.70710678118654752440);
  const T xa[3] = {T(P.xibar[0]) * s, T(P.xibar[1]) * s, T(P.xibar[2]) * s};
  const T r0 = T(P.rho0);
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const T gm = gam[x];
    const T c = gm + r0;
    T n2 = T(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const T zz = c * xa[q];
      zb[(size_t)q * g.N + x] = zz;
      zb[(size_t)(q + 3) * g.N + x] = zz;
      n2 += T(2) * zz * zz;
    }
    ab[x] = ball_scale(sqrt(n2), gm);
  }
}

// ---------------------------------------------------------------------------
// r = div^- A* w,  w = e^k - v^k / rho^k  (argument of the xi-step, eq:CCMF_FFT_ADMM):
// r[x] = (1/sqrt2) sum_c ( w1_c[x] + w2_c[x+e_c] - w1_c[x-e_c] - w2_c[x] ).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kUpd)
k_div(Geo g, const T* __restrict__ z, const T* __restrict__ a, T* __restrict__ r,
      const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  if (P.done) return;
  const T ir = T(1.0 / P.rho), irp = T(1.0 / P.rho_prev);
  const T* zb = z + (size_t)b * 6 * g.N;
  const T* ab = a + (size_t)b * g.N;
  T* rb = r + (size_t)b * g.N;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  for (int m = 0; m < g.tiles_per_blk; ++m) {
    const int t = tile_of(g, lb, m);
    if (t >= g.tiles) break;
    const uint32_t x = (uint32_t)t * kUpd + threadIdx.x;
    if (x >= g.N) continue;
    const Nbr nb = neighbours(g, x);
    const T bx = beta_of(ab[x], irp, ir);
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T w1 = bx * zb[(size_t)c * g.N + x];
      const T w2 = bx * zb[(size_t)(c + 3) * g.N + x];
      const T w2p = beta_of(ab[nb.p[c]], irp, ir) * zb[(size_t)(c + 3) * g.N + nb.p[c]];
      const T w1m = beta_of(ab[nb.m[c]], irp, ir) * zb[(size_t)c * g.N + nb.m[c]];
      acc += (w1 + w2p) - (w1m + w2);
    }
    rb[x] = acc * T(0.70710678118654752440);
  }
}

template <typename T>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Fused xi-step assembly, relaxation, ball projection, multiplier update and
// FP64 partial reductions (eq:CCMF_FFT_ADMM, second form; eq:convergence_criterion).
// With t_c[x] = xibar_c + phi[x+e_c] - phi[x] (= xibar + grad^+ phi):
//   xi^{k+1/2} = A(xibar + grad^+ phi) + (Id - A A*) w
//   xi1_c[x]  = t_c[x]/sqrt2     + (w1_c[x] - w2_c[x+e_c])/2
//   xi2_c[x]  = t_c[x-e_c]/sqrt2 + (w2_c[x] - w1_c[x-e_c])/2
//   xi^{k+1}  = 2(1-delta) xi^{k+1/2} - (1-2delta) e^k
//   z'        = v^k + rho^k xi^{k+1};  alpha' = min(1, gamma/|z'|)
// ---------------------------------------------------------------------------
// Each block walks g.tiles_per_blk tiles (see tile_of) and writes one FP64
// partial row, reduced by k_finish.
template <typename T>
__global__ void __launch_bounds__(kUpd)
k_update(Geo g, const T* __restrict__ kap, const T* __restrict__ z, const T* __restrict__ a,
         const double* __restrict__ phi, T* __restrict__ zn, T* __restrict__ an,
         double* __restrict__ partials, const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  if (P.done) return;
  const T rho = T(P.rho);
  const T ir = T(1.0 / P.rho), irp = T(1.0 / P.rho_prev);
  const T c_relax = T(2.0 * (1.0 - P.delta)), c_old = T(1.0 - 2.0 * P.delta);
  const T s = T(0.70710678118654752440);
  const T* gam = kap + (size_t)P.field * g.N;
  const T* zb = z + (size_t)b * 6 * g.N;
  const T* ab = a + (size_t)b * g.N;
  const double* pb = phi + (size_t)b * g.N;
  T* znb = zn + (size_t)b * 6 * g.N;
  T* anb = an + (size_t)b * g.N;

  double acc[kNQU];
#pragma unroll
  for (int q = 0; q < kNQU; ++q) acc[q] = 0.0;

  // Plane walk (g.tpp > 0): step m+1 visits the same in-plane tile one i-plane
  // further, so the x+e_1 values a thread loads at step m are its centre values
  // at step m+1, and its centre values at step m are its x-e_1 values at step
  // m+1.  They are carried in registers instead of being read again.
  const bool walk = g.tpp > 0;
  bool have = false;
  T nx_a = T(0), nx_z3 = T(0), pv_a = T(0), pv_z0 = T(0);
  double nx_ph = 0.0, pv_ph = 0.0;

  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  for (int m = 0; m < g.tiles_per_blk; ++m) {
    const int t = tile_of(g, lb, m);
    if (t >= g.tiles) break;
    const uint32_t x = (uint32_t)t * kUpd + threadIdx.x;
    if (x >= g.N) {
      have = false;
      continue;
    }
    const Nbr nb = neighbours(g, x);
    T zo[6], xh[6];
    T al, am0, z0m0;
    double ph, phm0;
    if (have) {
      al = nx_a;
      ph = nx_ph;
      zo[3] = nx_z3;
      am0 = pv_a;
      z0m0 = pv_z0;
      phm0 = pv_ph;
    } else {
      al = ab[x];
      ph = pb[x];
      zo[3] = zb[(size_t)3 * g.N + x];
      am0 = ab[nb.m[0]];
      z0m0 = zb[nb.m[0]];
      phm0 = pb[nb.m[0]];
    }
    const T bx = beta_of(al, irp, ir);
    const T gm = gam[x];
    zo[0] = zb[x];
    zo[1] = zb[(size_t)g.N + x];
    zo[2] = zb[(size_t)2 * g.N + x];
    zo[4] = zb[(size_t)4 * g.N + x];
    zo[5] = zb[(size_t)5 * g.N + x];
    const T ap0 = ab[nb.p[0]];
    const T z3p0 = zb[(size_t)3 * g.N + nb.p[0]];
    const double php0 = pb[nb.p[0]];
    {
      // c = 0 from the carried or freshly read x +- e_1 values
      const T w2p = beta_of(ap0, irp, ir) * z3p0;
      const T w1m = beta_of(am0, irp, ir) * z0m0;
      const T tp = T(P.xibar[0] + (php0 - ph));
      const T tm = T(P.xibar[0] + (ph - phm0));
      xh[0] = tp * s + T(0.5) * (bx * zo[0] - w2p);
      xh[3] = tm * s + T(0.5) * (bx * zo[3] - w1m);
    }
#pragma unroll
    for (int c = 1; c < 3; ++c) {
      const T w2p = beta_of(ab[nb.p[c]], irp, ir) * zb[(size_t)(c + 3) * g.N + nb.p[c]];
      const T w1m = beta_of(ab[nb.m[c]], irp, ir) * zb[(size_t)c * g.N + nb.m[c]];
      // xibar + grad^+ phi formed in FP64: phi is O(N), its differences O(1)
      const T tp = T(P.xibar[c] + (pb[nb.p[c]] - ph));
      const T tm = T(P.xibar[c] + (ph - pb[nb.m[c]]));
      xh[c] = tp * s + T(0.5) * (bx * zo[c] - w2p);
      xh[c + 3] = tm * s + T(0.5) * (bx * zo[c + 3] - w1m);
    }
    nx_a = ap0;
    nx_z3 = z3p0;
    nx_ph = php0;
    pv_a = al;
    pv_z0 = zo[0];
    pv_ph = ph;
    have = walk;
    const T ce = (T(1) - al) * irp;  // e^k = ce z, v^k = al z
    T d2 = T(0), xn2 = T(0), zn2 = T(0);
    T zz[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const T e = ce * zo[q];
      const T v = al * zo[q];
      const T d = e - xh[q];
      d2 += d * d;
      xn2 += xh[q] * xh[q];
      acc[Q_MV + q] += (double)v;
      const T x1 = c_relax * xh[q] - c_old * e;
      zz[q] = v + rho * x1;
      zn2 += zz[q] * zz[q];
    }
    acc[Q_RES2] += (double)d2;
    acc[Q_E] += (double)(gm * sqrt(xn2));
    const T aln = ball_scale(sqrt(zn2), gm);
    const T cen = (T(1) - aln) * ir;
    double bbn = 0.0, bbd = 0.0, vv = 0.0, ee = 0.0, dvv = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      znb[(size_t)q * g.N + x] = zz[q];
      const double vn = (double)(aln * zz[q]);
      const double en = (double)(cen * zz[q]);
      const double dv = vn - (double)(al * zo[q]);
      const double de = en - (double)(ce * zo[q]);
      bbn += dv * de;
      bbd += de * de;
      dvv += dv * dv;
      vv += vn * vn;
      ee += en * en;
    }
    anb[x] = aln;
    acc[Q_BBN] += bbn;
    acc[Q_BBD] += bbd;
    acc[Q_VV] += vv;
    acc[Q_EE] += ee;
    acc[Q_DVV] += dvv;
    double du = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) du += P.xibar[c] * (double)(al * (zo[c] + zo[c + 3]));
    acc[Q_DUAL] += du * 0.70710678118654752440;
  }

  // deterministic block reduction: wavefront shuffles, then fixed-order LDS sum
  __shared__ double red[kUpd / 64][kNQU];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kNQU; ++q) {
    const double sq = wave_sum<T>(acc[q]);
    if (lane == 0) red[wv][q] = sq;
  }
  __syncthreads();
  if (threadIdx.x < kNQ) {   // whole row, unused columns zero
    double sq = 0.0;
    if (threadIdx.x < kNQU) {
#pragma unroll
      for (int w = 0; w < kUpd / 64; ++w) sq += red[w][threadIdx.x];
    }
    partials[((size_t)b * gridDim.x + lb) * kNQ + threadIdx.x] = sq;
  }
}

// ---------------------------------------------------------------------------
// Fixed-order sum of `nrows` partial rows of kNQ doubles by a block of NT
// threads, read as one contiguous array so every wavefront load is coalesced:
// thread t always takes column t % kNQ, rows in increasing order; lanes of one
// column are combined by shuffles and the wavefronts in order.  Result in
// out[0..kNQU) of the shared array (valid after the call for all threads).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void block_sum_rows(const double* __restrict__ rows, int nrows, double* out) {
  static_assert(NT % 64 == 0 && kNQ == 16, "layout");
  __shared__ double red[NT / 64][kNQ];
  double acc = 0.0;
  const int total = nrows * kNQ;
  // U rows of loads in flight, added in the same order as one row at a time
  constexpr int U = 16;
  int e = threadIdx.x;
  for (; e + (U - 1) * NT < total; e += U * NT) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = rows[e + u * NT];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; e < total; e += NT) acc += rows[e];
  acc += __shfl_down(acc, 32, 64);
  acc += __shfl_down(acc, 16, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane < kNQ) red[wv][lane] = acc;
  __syncthreads();
  if (threadIdx.x < kNQ) {
    double sq = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) sq += red[w][threadIdx.x];
    out[threadIdx.x] = sq;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Per-problem reduction of the partials in a fixed order, the stopping test of
// eq:convergence_criterion and the adaptive penalty of Sec. 3.2 (device side, no
// host round trip).  One block per problem.
// ---------------------------------------------------------------------------
constexpr int kFinishThreads = 1024;

__global__ void __launch_bounds__(kFinishThreads)
k_finish(uint32_t N, int nparts, const double* __restrict__ partials, Prob* __restrict__ prob,
         double* __restrict__ hist, int hist_len) {
  const int b = blockIdx.x;
  Prob& P = prob[b];
  if (P.done) return;
  // the iteration index lives on the device, so a captured chunk of iterations
  // can be replayed unchanged
  const int it = P.k;
  __shared__ double red[1][kNQ];
  block_sum_rows<kFinishThreads>(partials + (size_t)b * nparts * kNQ, nparts, red[0]);
  if (threadIdx.x != 0) return;
  const double invN = 1.0 / (double)N;
  const double res = sqrt(red[0][Q_RES2] * invN);
  double mv2 = 0.0;
  for (int q = 0; q < 6; ++q) {
    const double m = red[0][Q_MV + q] * invN;
    mv2 += m * m;
  }
  const double mvn = sqrt(mv2);
  const double E = red[0][Q_E] * invN;
  if (hist != nullptr && it < hist_len) {
    double* h = hist + ((size_t)b * hist_len + it) * 4;
    h[0] = res;
    h[1] = P.rho;
    h[2] = E;
    h[3] = mvn;
  }
  const bool conv = (res <= P.tol * mvn) || P.all_zero;
  if (conv || it + 1 >= P.max_iter) {
    P.geff = E;
    P.res = res;
    P.mvn = mvn;
    P.dual = red[0][Q_DUAL] * invN;
    // <A* v>_c = (<v1_c> + <v2_c>) / sqrt(2): the shift in A* leaves the mean unchanged
    for (int c = 0; c < 3; ++c)
      P.mflux[c] = (red[0][Q_MV + c] + red[0][Q_MV + 3 + c]) * invN * 0.70710678118654752440;
    P.done = conv ? 1 : 2;
    P.k = it;
    return;
  }
  // adaptive penalty of Sec. 3.2 with the safeguard (rule codes of include/ccmf.h)
  double cand = -1.0;
  const double vv = red[0][Q_VV], ee = red[0][Q_EE];
  const double ltd = (vv > 0.0 && ee > 0.0) ? sqrt(vv / ee) : -1.0;
  if (P.rule == 0) {  // Barzilai-Borwein, reliable estimates only, else Lorenz-Tran-Dinh
    const double num = red[0][Q_BBN], den = red[0][Q_BBD], dvv = red[0][Q_DVV];
    cand = (num > 0.0 && den > 0.0 && num >= P.bb_corr * sqrt(den * dvv)) ? num / den : ltd;
  } else if (P.rule == 2) {  // Lorenz-Tran-Dinh
    cand = ltd;
  }
  double rn = P.rho;
  if (cand > 0.0 && isfinite(cand)) {
    const double q = 1.0 + (double)(it + P.k_off) / P.k0;
    const double grow = 1.0 + P.eta0 / (q * q);   // summable relative variation
    rn = fmin(fmax(cand, P.rho / grow), P.rho * grow);
    rn = fmin(fmax(rn, P.lo), P.hi);
  }
  P.rho_prev = P.rho;
  P.rho = rn;
  P.k = it + 1;
}

// ---------------------------------------------------------------------------
// Outputs at the stopping iterate
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_flux(Geo g, const T* __restrict__ z0, const T* __restrict__ z1, const T* __restrict__ a0,
       const T* __restrict__ a1, T* __restrict__ flux, const Prob* __restrict__ prob) {
  // face fluxes A* v = (v1 + S* v2)/sqrt2 (eq:CCMF_FFT_AOperator_adjoint), v = alpha z
  const int b = blockIdx.y;
  const int par = prob[b].k & 1;
  const T* zb = (par ? z1 : z0) + (size_t)b * 6 * g.N;
  const T* ab = (par ? a1 : a0) + (size_t)b * g.N;
  T* fb = flux + (size_t)b * 3 * g.N;
  const T s = T(0.70710678118654752440);
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const Nbr nb = neighbours(g, x);
    const T al = ab[x];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      fb[(size_t)c * g.N + x] =
          s * (al * zb[(size_t)c * g.N + x] + ab[nb.p[c]] * zb[(size_t)(c + 3) * g.N + nb.p[c]]);
  }
}

// Checkpoint: v^k = alpha z and e^k = (1 - alpha) z / rho^{k-1} of the stopping state
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_get_state(Geo g, const T* __restrict__ z0, const T* __restrict__ z1, const T* __restrict__ a0,
            const T* __restrict__ a1, T* __restrict__ v, T* __restrict__ e, const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  const int par = P.k & 1;
  const T* zb = (par ? z1 : z0) + (size_t)b * 6 * g.N;
  const T* ab = (par ? a1 : a0) + (size_t)b * g.N;
  const T irp = T(1.0 / P.rho_prev);
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const T al = ab[x];
    const T ce = (T(1) - al) * irp;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const T zq = zb[(size_t)q * g.N + x];
      if (v) v[((size_t)b * 6 + q) * g.N + x] = al * zq;
      if (e) e[((size_t)b * 6 + q) * g.N + x] = ce * zq;
    }
  }
}

// Warm start from a pair (v, e): with rho = rho^k (the plan sets rho^{k-1} = rho^k)
// z = v + rho e and alpha = |v|/|z| reproduce v = alpha z and e = (1 - alpha) z / rho
// exactly when v and e are non-negative multiples of one vector at every voxel, as
// every ADMM iterate is.  Per block: number of voxels violating that (or not finite).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_set_state(Geo g, const T* __restrict__ v, const T* __restrict__ e, T* __restrict__ z, T* __restrict__ a,
            double* __restrict__ partials, const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const double rho = prob[b].rho;
  const T* vb = v + (size_t)b * 6 * g.N;
  const T* eb = e + (size_t)b * 6 * g.N;
  T* zb = z + (size_t)b * 6 * g.N;
  T* ab = a + (size_t)b * g.N;
  int bad = 0;
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    double vv = 0.0, ee = 0.0, ve = 0.0, zz = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double vq = (double)vb[(size_t)q * g.N + x], eq = (double)eb[(size_t)q * g.N + x];
      const double zq = vq + rho * eq;
      zb[(size_t)q * g.N + x] = T(zq);
      vv += vq * vq;
      ee += eq * eq;
      ve += vq * eq;
      zz += zq * zq;
    }
    const double nv = sqrt(vv), nz = sqrt(zz);
    ab[x] = nz > 0.0 ? T(fmin(1.0, nv / nz)) : T(1);
    const bool ok = isfinite(zz) && (nv * sqrt(ee) - ve <= 1e-6 * nv * sqrt(ee));
    bad += ok ? 0 : 1;
  }
  __shared__ int cnt[kThreads];
  cnt[threadIdx.x] = bad;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[((size_t)b * gridDim.x + blockIdx.x) * kNQ] = (double)cnt[0];
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_grad(Geo g, const T* __restrict__ z0, const T* __restrict__ z1, const T* __restrict__ a0,
       const T* __restrict__ a1, const double* __restrict__ phi, const double* __restrict__ dl,
       T* __restrict__ dkap, const Prob* __restrict__ prob) {
  // d geff / d gamma[x] = |xi^{k+1/2}[x]| / N, xi^{k+1/2} rebuilt from the stopping state
  const int f = blockIdx.y;
  const T s = T(0.70710678118654752440);
  const T invN = T(1.0 / (double)g.N);
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const Nbr nb = neighbours(g, x);
    T out = T(0);
    for (int l = 0; l < g.nloads; ++l) {
      const int b = f * g.nloads + l;
      const Prob& P = prob[b];
      const int par = P.k & 1;
      const T* zb = (par ? z1 : z0) + (size_t)b * 6 * g.N;
      const T* ab = (par ? a1 : a0) + (size_t)b * g.N;
      const double* pb = phi + (size_t)b * g.N;
      const T ir = T(1.0 / P.rho), irp = T(1.0 / P.rho_prev);
      const T bx = beta_of(ab[x], irp, ir);
      const double ph = pb[x];
      T xn2 = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T w2p = beta_of(ab[nb.p[c]], irp, ir) * zb[(size_t)(c + 3) * g.N + nb.p[c]];
        const T w1m = beta_of(ab[nb.m[c]], irp, ir) * zb[(size_t)c * g.N + nb.m[c]];
        const T x1 = T(P.xibar[c] + (pb[nb.p[c]] - ph)) * s + T(0.5) * (bx * zb[(size_t)c * g.N + x] - w2p);
        const T x2 = T(P.xibar[c] + (ph - pb[nb.m[c]])) * s + T(0.5) * (bx * zb[(size_t)(c + 3) * g.N + x] - w1m);
        xn2 += x1 * x1 + x2 * x2;
      }
      out += T(dl[b]) * sqrt(xn2) * invN;
    }
    dkap[(size_t)f * g.N + x] = out;
  }
}

// kappa statistics for validation and the penalty window: per block
// (min positive, max, count of negative or non-finite entries)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_kappa_stats(const T* __restrict__ kap, uint32_t N, double* __restrict__ out) {
  const int f = blockIdx.y;
  const T* gk = kap + (size_t)f * N;
  double mn = INFINITY, mx = 0.0, bad = 0.0;
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < N; x += gridDim.x * kThreads) {
    const double v = (double)gk[x];
    if (!(v >= 0.0) || !isfinite(v)) {
      bad += 1.0;
      continue;
    }
    if (v > 0.0 && v < mn) mn = v;
    if (v > mx) mx = v;
  }
  __shared__ double s[3][kThreads];
  s[0][threadIdx.x] = mn;
  s[1][threadIdx.x] = mx;
  s[2][threadIdx.x] = bad;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = out + ((size_t)f * gridDim.x + blockIdx.x) * 3;
    o[0] = s[0][0];
    o[1] = s[1][0];
    o[2] = s[2][0];
  }
}

// ---------------------------------------------------------------------------
// Certified dual bound (strong duality, Sec. 2.1; max-flow form eq:CCMF_FFT_problemA).
// y = A* v is a face flux; y_df = y - grad^+ L^dagger div^- y is divergence free with
// the same mean, so y_df / max(1, sigma), sigma = max |A y_df| / gamma, is feasible
// and <xibar, y>/max(1, sigma) <= geff.  k_cert_r forms div^- y, k_cert_sigma the max.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cert_r(Geo g, const T* __restrict__ z0, const T* __restrict__ z1, const T* __restrict__ a0,
         const T* __restrict__ a1, T* __restrict__ r, const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const int par = prob[b].k & 1;
  const T* zb = (par ? z1 : z0) + (size_t)b * 6 * g.N;
  const T* ab = (par ? a1 : a0) + (size_t)b * g.N;
  T* rb = r + (size_t)b * g.N;
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const Nbr nb = neighbours(g, x);
    const T ax = ab[x];
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // y_c[x] - y_c[x - e_c] with y_c[x] = (v_c[x] + v_{3+c}[x + e_c]) / sqrt2
      const T v1 = ax * zb[(size_t)c * g.N + x];
      const T v2 = ax * zb[(size_t)(c + 3) * g.N + x];
      const T v2p = ab[nb.p[c]] * zb[(size_t)(c + 3) * g.N + nb.p[c]];
      const T v1m = ab[nb.m[c]] * zb[(size_t)c * g.N + nb.m[c]];
      acc += (v1 + v2p) - (v1m + v2);
    }
    rb[x] = acc * T(0.70710678118654752440);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cert_sigma(Geo g, const T* __restrict__ kap, const T* __restrict__ z0, const T* __restrict__ z1,
             const T* __restrict__ a0, const T* __restrict__ a1, const double* __restrict__ phic,
             double* __restrict__ out, const Prob* __restrict__ prob) {
  const int b = blockIdx.y;
  const Prob& P = prob[b];
  const int par = P.k & 1;
  const T* zb = (par ? z1 : z0) + (size_t)b * 6 * g.N;
  const T* ab = (par ? a1 : a0) + (size_t)b * g.N;
  const T* gam = kap + (size_t)P.field * g.N;
  const double* pb = phic + (size_t)b * g.N;
  const double s = 0.70710678118654752440;
  double mx = 0.0, bad = 0.0, ynorm = 0.0;
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < g.N; x += gridDim.x * kThreads) {
    const Nbr nb = neighbours(g, x);
    const double ax = (double)ab[x];
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // face c of x (y_df_c[x]) and face c of x - e_c (y_df_c[x - e_c])
      const double yx = s * (ax * (double)zb[(size_t)c * g.N + x] +
                             (double)ab[nb.p[c]] * (double)zb[(size_t)(c + 3) * g.N + nb.p[c]]);
      const double ym = s * ((double)ab[nb.m[c]] * (double)zb[(size_t)c * g.N + nb.m[c]] +
                             ax * (double)zb[(size_t)(c + 3) * g.N + x]);
      const double fx = yx - (pb[nb.p[c]] - pb[x]);
      const double fm = ym - (pb[x] - pb[nb.m[c]]);
      n2 += 0.5 * (fx * fx + fm * fm);
    }
    const double nrm = sqrt(n2);
    const double gm = (double)gam[x];
    if (gm > 0.0) {
      mx = fmax(mx, nrm / gm);
    } else {
      bad = fmax(bad, nrm);
    }
    ynorm = fmax(ynorm, nrm);
  }
  __shared__ double red[3][kThreads];
  red[0][threadIdx.x] = mx;
  red[1][threadIdx.x] = bad;
  red[2][threadIdx.x] = ynorm;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[((size_t)b * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kThreads)
k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

}  // namespace ccmf
