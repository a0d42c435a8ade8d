// HIP kernels for gfx950 (64-lane wavefronts): the fine five-point operator,
// the batched block-LDL^T box solves of the MRCM-OS apply, the level-scheduled
// coarse interface solve, multiscale reconstruction, Schwarz smoothing and the
// fused Arnoldi vector kernels of GMRES.  Every reduction has a fixed order,
// so results are bit-identical from run to run.
#include <type_traits>

#include "device.h"
#include "internal.h"

namespace mrcm {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of kVecThreads threads; result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) s += red[k];
  return s;
}

// Sum of nb partials, identical order in every block.
// Elements a thread handles per round of a grid-stride loop: the loads of a
// round are all issued (indices clamped into range) before any is used, so
// they are in flight together; a thread still visits its elements in
// increasing order, so the reductions keep one fixed order.
constexpr int kRound = 4;

__device__ __forceinline__ double reduce_partials(const double* part, int nb, double* red) {
  double v = 0.0;
  for (int k0 = threadIdx.x; k0 < nb; k0 += kRound * blockDim.x) {
    double a[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const int k = k0 + u * blockDim.x;
      a[u] = part[k < nb ? k : nb - 1];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
      if (k0 + u * (int)blockDim.x < nb) v += a[u];
  }
  return block_sum(v, red);
}

// y_c = sum_f t_f (x_c - x_c') over the four faces; boundary faces carry the
// Dirichlet half-transmissibility (coupled to zero) or zero.  Branch-free:
// missing neighbours are read at the cell itself and meet a zero
// coefficient, so all loads are unconditional.
template <typename T>
__device__ __forceinline__ T stencil(const T* __restrict__ tx, const T* __restrict__ ty, int nx,
                                     int ny, int ix, int iy, const T* __restrict__ x) {
  const long long c = (long long)iy * nx + ix;
  const long long fx = (long long)iy * (nx + 1) + ix;
  const T tW = tx[fx], tE = tx[fx + 1], tS = ty[c], tN = ty[c + nx];
  const T xc = x[c];
  const T xw = x[ix > 0 ? c - 1 : c], xe = x[ix + 1 < nx ? c + 1 : c];
  const T xs = x[iy > 0 ? c - nx : c], xn = x[iy + 1 < ny ? c + nx : c];
  T v = (tW + tE + tS + tN) * xc;
  v -= (ix > 0 ? tW : T(0)) * xw;
  v -= (ix + 1 < nx ? tE : T(0)) * xe;
  v -= (iy > 0 ? tS : T(0)) * xs;
  v -= (iy + 1 < ny ? tN : T(0)) * xn;
  return v;
}

__global__ void __launch_bounds__(kVecThreads) k_op_apply(const double* __restrict__ tx,
                                                          const double* __restrict__ ty, int nx,
                                                          int ny, const double* __restrict__ x,
                                                          double* __restrict__ y) {
  const long long n = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    y[c] = stencil(tx, ty, nx, ny, ix, iy, x);
  }
}

__global__ void k_rhs(const double* __restrict__ tx, const double* __restrict__ ty, int nx,
                      int ny, int bcW, int bcE, int bcS, int bcN, const double* __restrict__ f,
                      const double* __restrict__ g, double h, double* __restrict__ b) {
  const long long n = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    double v = f ? f[c] * h * h : 0.0;
    if (g) {
      if (ix == 0 && bcW) v += tx[(long long)iy * (nx + 1)] * g[iy];
      if (ix == nx - 1 && bcE) v += tx[(long long)iy * (nx + 1) + nx] * g[ny + iy];
      if (iy == 0 && bcS) v += ty[ix] * g[2 * ny + ix];
      if (iy == ny - 1 && bcN) v += ty[(long long)ny * nx + ix] * g[2 * ny + nx + ix];
    }
    b[c] = v;
  }
}

// Virtual block of a launch: its index and the block count of its grid.  A
// launch over one context uses the hardware grid; a launch over several
// contexts gives every column its own range of workgroups, each of which
// runs as block `id` of a grid of `n`, so that every column's arithmetic and
// reduction order are those of its own launch.
struct Blk {
  int id, n;
};
__device__ __forceinline__ Blk hw_blk() { return Blk{(int)blockIdx.x, (int)gridDim.x}; }

// ---- batched box solves ---------------------------------------------------
// One lane group of GS lanes (GS = 16, 32 or 64 >= the box width bx, 64 / GS
// boxes per wave) solves one cell box with the block LDL^T factor of its cell
// rows.  Lane r owns cell column r of every row j:
//   forward  u_j = D_j^-1 (b_j + T_j u_{j-1}),
//   backward x_j = u_j + D_j^-1 (T_{j+1} x_{j+1}).
// The blocks are symmetric and stored as half blocks (setup_jobs.h): lane r
// loads the entries D(r, r + k), k = 0 .. NB / 2, of each block and fetches
// D(r, r - k) = D(r - k, r) from the registers of lane r - k.  All exchange
// between the lanes of a group is wave-local (no workgroup barrier): the
// vector of a step goes through the group's slot of LDS, the mirrored
// entries through cross-lane permutes.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// a * b + c with one rounding, spelled out so that the one-RHS and the
// multi-RHS kernels round every step the same way whatever the optimiser
// would contract.
__device__ __forceinline__ float fmat(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fmat(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// Four consecutive words of a factor block (16 bytes of FP32 or 32 bytes of
// FP64), as native vectors the optimiser keeps in registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename S> struct Quad;
template <> struct Quad<float> {
  f32x4 v;
  __device__ float operator[](int i) const { return v[i]; }
};
template <> struct Quad<double> {
  f64x2 lo, hi;
  __device__ double operator[](int i) const { return i < 2 ? lo[i] : hi[i - 2]; }
};
__device__ __forceinline__ void load_quad(Quad<float>& q, const float* p) {
  q.v = *reinterpret_cast<const f32x4*>(p);
}
__device__ __forceinline__ void load_quad(Quad<double>& q, const double* p) {
  q.lo = *reinterpret_cast<const f64x2*>(p);
  q.hi = *reinterpret_cast<const f64x2*>(p + 2);
}

// Make v opaque to the optimiser at this point, so that addresses derived
// from it are recomputed here instead of being hoisted out of the row loop
// into registers for the whole kernel.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Shape of the half blocks of a launch of column width NB: rows 0 .. H, the
// first K0 of them single words, the others NH quads.
template <int NB>
struct Half {
  static constexpr int H = NB / 2;
  static constexpr int K0 = half_k0(NB);
  static constexpr int NH = half_quads(NB);
};

// A lane's rows of one half block.  row(k) is entry D(r, r + k) of lane r
// (k a constant after unrolling).
template <typename S, int NB>
struct HalfRow {
  Quad<S> q[Half<NB>::NH];
  S h[Half<NB>::K0 > 0 ? Half<NB>::K0 : 1];
  __device__ S row(int k) const {
    constexpr int K0 = Half<NB>::K0;
    return k < K0 ? h[k] : q[(k - K0) >> 2][(k - K0) & 3];
  }
};

// The largest power of two <= d, between 2 and 8.  A sweep runs its step
// count rounded up to a multiple of the depth, and powers of two divide the
// common box heights (16, 20, 32, 36 rows), where a depth of 5 would run 20
// steps for 16 rows.
constexpr int pow2_depth(int d) { return d >= 8 ? 8 : d >= 4 ? 4 : 2; }

// Blocks in flight per lane: as many as about 48 VGPRs of rows hold (more
// would cost waves per SIMD: a sweep over 48, 64, 80 and 96 found 48 and 64
// equal, 96 a third slower on 36-wide patches).
template <typename S, int NB>
constexpr int reg_depth() {
  constexpr int per_block = half_rows(NB) * (int)sizeof(S) / 4;
  return pow2_depth(48 / per_block);
}

// Lane rc's rows of one block of a box n cells wide: the quads at words
// (q n + rc) 4, the single words at 4 NH n + k n + rc, so the group reads
// contiguous pieces.
template <typename S, int NB>
__device__ __forceinline__ void load_half(HalfRow<S, NB>& d, const S* __restrict__ blk, int n,
                                          int rc) {
  constexpr int NH = Half<NB>::NH, K0 = Half<NB>::K0;
  const S* p = blk + 4 * rc;
#pragma unroll
  for (int q = 0; q < NH; ++q) load_quad(d.q[q], p + (long long)q * 4 * n);
  const S* t = blk + (long long)4 * NH * n + rc;
#pragma unroll
  for (int k = 0; k < K0; ++k) d.h[k] = t[(long long)k * n];
}

// Value v of the lane whose byte address (4 x lane index) is addr.
__device__ __forceinline__ float lane_fetch(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(int addr, double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Byte addresses of the lanes that hold D(rc, rc - k), k = 1 .. H: lane
// (rc - k) mod n of the group starting at lane g0 (lane g0 for k > n, where
// every lane holds a zero row), one byte each, four to a word.
template <int H>
__device__ __forceinline__ void mirror_lanes(int (&src)[(H + 3) / 4], int g0, int rc, int n) {
#pragma unroll
  for (int w = 0; w < (H + 3) / 4; ++w) src[w] = 0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    int c = rc - k;
    c = c < 0 ? c + n : c;
    c = c < 0 ? 0 : c;
    src[(k - 1) >> 2] |= (4 * (g0 + c)) << (8 * ((k - 1) & 3));
  }
}

// The mirrored entries rot[k - 1] = D(rc, rc - k) of one block.  The packed
// addresses are unpacked at each use (opaque keeps the optimiser from
// holding all H of them in registers across the sweep).
template <typename S, int NB>
__device__ __forceinline__ void mirror_rows(S (&rot)[Half<NB>::H], const HalfRow<S, NB>& d,
                                            const int (&src)[(Half<NB>::H + 3) / 4]) {
  int w[(Half<NB>::H + 3) / 4];
#pragma unroll
  for (int i = 0; i < (Half<NB>::H + 3) / 4; ++i) w[i] = opaque(src[i]);
#pragma unroll
  for (int k = 1; k <= Half<NB>::H; ++k)
    rot[k - 1] = lane_fetch((w[(k - 1) >> 2] >> (8 * ((k - 1) & 3))) & 255, d.row(k));
}

// acc = sum_c D(rc, c) v[c]: the lane's rows k against vo[k] = v[(rc + k)
// mod n], the mirrored entries against vr[-k] = v[(rc - k) mod n] (vo and vr
// point into the group's doubled copy of v); four partial sums shorten the
// chain of dependent additions.
template <typename T, typename S, int NB>
__device__ __forceinline__ T half_dot(const HalfRow<S, NB>& d, const S (&rot)[Half<NB>::H],
                                      const T* vo, const T* vr) {
  constexpr int NH = Half<NB>::NH, K0 = Half<NB>::K0, H = Half<NB>::H;
  T a[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < NH; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = fmat((T)d.q[q][i], vo[K0 + 4 * q + i], a[i]);
#pragma unroll
  for (int k = 0; k < K0; ++k) a[k] = fmat((T)d.h[k], vo[k], a[k]);
#pragma unroll
  for (int k = 1; k <= H; ++k) a[(k - 1) & 3] = fmat((T)rot[k - 1], vr[-k], a[(k - 1) & 3]);
  return (a[0] + a[1]) + (a[2] + a[3]);
}

// Largest value of v over the 64 lanes of the wave, as a wave-uniform value.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// One sweep over the block rows of the boxes of a wave.  Step s uses block
// blk(s), whose rows were loaded into register set s % DEPTH at step
// s - DEPTH; right after its use the set is refilled with block s + DEPTH,
// so every block has DEPTH - 1 steps to arrive.  The boxes of a wave have
// different heights, so the wave runs nmax steps (its largest count, rounded
// up to a multiple of DEPTH); a group's steps past its own nsteps re-load its
// last block and are told valid = false.  No load is conditional, so the
// compiler counts the loads in flight exactly and waits only for the block
// a step uses (an early exit from the unrolled steps instead of the rounding
// made the compiler wait for more loads and was slower).
template <typename S, int NB, int DEPTH, typename Blk, typename Step>
__device__ __forceinline__ void pipelined_sweep(int nsteps, int nmax, Blk blk, Step step,
                                                const S* __restrict__ Dinv, int bstride,
                                                int n, int r) {
  const int last = nsteps > 0 ? nsteps - 1 : 0;
  auto src = [&](int s) {
    const int b = blk(s < last ? s : last);
    return Dinv + (long long)(b > 0 ? b : 0) * bstride;
  };
  HalfRow<S, NB> reg[DEPTH];
#pragma unroll
  for (int u = 0; u < DEPTH; ++u) load_half<S, NB>(reg[u], src(u), n, opaque(r));
  for (int s0 = 0; s0 < nmax; s0 += DEPTH) {
#pragma unroll
    for (int u = 0; u < DEPTH; ++u) {
      const int s = s0 + u;
      step(s, reg[u], s < nsteps);
      load_half<S, NB>(reg[u], src(s + DEPTH), n, opaque(r));
    }
  }
}

// Steps a wave runs for the largest of n over its groups: rounded up to a
// multiple of DEPTH.
template <int DEPTH>
__device__ __forceinline__ int wave_steps(int n) {
  const int m = wave_max(n);
  return (m + DEPTH - 1) / DEPTH * DEPTH;
}

// Words of the group's copy of the step vector for column width NB and group
// size GS: v at [H, H + n) and again at [H + n, H + 2 n), zeros around it
// (the lane's rows past the box meet finite values).
template <int NB, int GS>
constexpr int vec_words() { return (NB / 2 + 2 * GS + 3) / 4 * 4; }

// Zero the group's vector slots (count words) before the first step.
template <typename T, int GS>
__device__ __forceinline__ void zero_slots(T* v, int count, int lane) {
  for (int i = lane; i < count; i += GS) v[i] = T(0);
}

// Block LDL^T solve of one box by a group; us holds b on entry and x on exit
// in rows stop .. by - 1 (by rows of bx words, LDS; the backward pass ends at
// row stop, the first row the caller reads, and rows below it keep their
// forward values); cp holds the couplings T_j (LDS); vv is the group's vector
// slot (vec_words, zeroed); g0 the group's first lane in the wave.  S is the storage type of the factors, T the arithmetic and vector
// type (FP32 factors may be applied in FP64 arithmetic).  Lanes at or past
// bx (and whole groups with live = false) take part in every step but read
// only inside the box and write nothing outside their slot.
template <typename T, typename S, int NB, int GS>
__device__ __forceinline__ void box_solve(T* us, T* vv, const S* cp, const S* __restrict__ Dinv,
                                          int bx, int by, int bstride, int r, int g0,
                                          bool live, int stop) {
  constexpr int H = Half<NB>::H;
  constexpr int DEPTH = reg_depth<S, NB>();
  const bool act = live && r < bx;
  const int rc = r < bx ? r : bx - 1;
  int src[(H + 3) / 4];
  mirror_lanes<H>(src, g0, rc, bx);
  const T* vo = vv + H + rc;
  const T* vr = vv + H + rc + bx;
  T carry = T(0);
  pipelined_sweep<S, NB, DEPTH>(
      live ? by : 0, wave_steps<DEPTH>(live ? by : 0), [](int s) { return s; },
      [&](int s, const HalfRow<S, NB>& d, bool valid) {
        S rot[H];
        mirror_rows<S, NB>(rot, d, src);
        const int j = s < by ? s : by - 1;
        const T uj = us[j * bx + rc];
        const T y = j > 0 ? fmat((T)cp[j * bx + rc], carry, uj) : uj;
        const bool w = act && valid;
        if (r < bx) vv[H + r] = vv[H + bx + r] = w ? y : T(0);
        wave_sync();
        const T acc = half_dot<T, S, NB>(d, rot, vo, vr);
        wave_sync();
        if (w) us[j * bx + r] = acc;
        carry = w ? acc : carry;
      },
      Dinv, bstride, bx, rc);
  // carry = x_{by-1} = u_{by-1}; rows by - 2 down to stop
  const int nb = live && by - 1 - stop > 0 ? by - 1 - stop : 0;
  pipelined_sweep<S, NB, DEPTH>(
      nb, wave_steps<DEPTH>(nb), [by](int s) { return by - 2 - s; },
      [&](int s, const HalfRow<S, NB>& d, bool valid) {
        S rot[H];
        mirror_rows<S, NB>(rot, d, src);
        int j = by - 2 - s;
        j = j < 0 ? 0 : j;
        const int jn = j + 1 < by ? j + 1 : by - 1;
        const bool w = act && valid;
        const T y = (T)cp[jn * bx + rc] * carry;
        if (r < bx) vv[H + r] = vv[H + bx + r] = w ? y : T(0);
        wave_sync();
        const T acc = half_dot<T, S, NB>(d, rot, vo, vr);
        wave_sync();
        const T xj = us[j * bx + rc] + acc;
        if (w) us[j * bx + r] = xj;
        carry = w ? xj : carry;
      },
      Dinv, bstride, bx, rc);
}

// Stage a box for its solve: rows [0, by) of a grid vector (bx cells wide,
// lane r: column r) and the box's couplings (by rows of bx words) into LDS,
// sixteen rows of both in flight at a time, so that a box of up to sixteen
// rows costs one memory latency.  Loads are unconditional (row and column
// clamped into the box); the wave runs the rows of its tallest box.
template <typename T, typename G, typename S>
__device__ __forceinline__ void stage_box(T* dst, const G* __restrict__ src, long long origin,
                                          int nx, S* cdst, const S* __restrict__ csrc, int bx,
                                          int by, int lane, bool live) {
  const int rows = wave_max(live ? by : 0);
  const int col = lane < bx ? lane : bx - 1;
  const bool act = live && lane < bx;
  for (int j0 = 0; j0 < rows; j0 += 16) {
    G v[16];
    S c[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + u < by ? j0 + u : by - 1;
      v[u] = src[origin + (long long)j * nx + col];
      c[u] = csrc[j * bx + col];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (act && j0 + u < by) {
        dst[(j0 + u) * bx + lane] = (T)v[u];
        cdst[(j0 + u) * bx + lane] = c[u];
      }
  }
}

// Copy count (>= 1) contiguous words from global memory into LDS with the
// whole group, eight unconditional loads in flight per lane at a time.
template <typename S, int GS>
__device__ __forceinline__ void words_to_lds(S* dst, const S* __restrict__ src, int count,
                                             int lane, bool live) {
  const int total = wave_max(live ? count : 0);
  for (int q0 = 0; q0 < total; q0 += 8 * GS) {
    S v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * GS + lane;
      v[u] = src[q < count ? q : count - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * GS + lane;
      if (live && q < count) dst[q] = v[u];
    }
  }
}

// LDS slot of one lane group:
//   vv[vec_words] (T) | cp[max cells] (S) | us[max cells] (T),
// every part 16-byte aligned; cp_words (the coupling area) is a multiple of
// 16 bytes.
template <typename T, typename S, int NB, int GS>
struct BoxSlot {
  T* vv;
  S* cp;
  T* us;
  __device__ BoxSlot(char* base, int cp_words) {
    constexpr int VW = vec_words<NB, GS>();
    vv = reinterpret_cast<T*>(base);
    cp = reinterpret_cast<S*>(base + VW * sizeof(T));
    us = reinterpret_cast<T*>(base + VW * sizeof(T) + (long long)cp_words * sizeof(S));
  }
};

// Legendre polynomial P_q at the face parameter xi_j = (2 j + 1) / n - 1
// (three-term recurrence).
__device__ __forceinline__ double legendre_face(int q, int j, int n) {
  const double xi = (2.0 * j + 1.0) / n - 1.0;
  double pm = 1.0, pq = xi;
  if (q == 0) return 1.0;
  for (int k = 1; k < q; ++k) {
    const double pn = ((2.0 * k + 1.0) * xi * pq - k * pm) / (k + 1.0);
    pm = pq;
    pq = pn;
  }
  return pq;
}

// Box-local indices (row stride d.bx) of the two cells of face j of side
// `side` (W E S N) of the owned subdomain of box d: the subdomain's cell and
// the cell across the face.  A face on the box's boundary (no oversampling)
// has no cell across inside the box; its second index is the first (the
// weights of that cell are zero).
__device__ __forceinline__ void face_cells(const BoxDesc& d, int side, int j, int& cin,
                                           int& cout) {
  int row, col, dr = 0, dc = 0;
  if (side == 0) {
    row = d.oy + j; col = d.ox; dc = -1;
  } else if (side == 1) {
    row = d.oy + j; col = d.ox + d.obx - 1; dc = 1;
  } else if (side == 2) {
    row = d.oy; col = d.ox + j; dr = -1;
  } else {
    row = d.oy + d.oby - 1; col = d.ox + j; dr = 1;
  }
  cin = row * d.bx + col;
  const int r2 = row + dr, c2 = col + dc;
  cout = (r2 < 0 || r2 >= d.by || c2 < 0 || c2 >= d.bx) ? cin : r2 * d.bx + c2;
}

// Flux and pressure moments of one coarse dof k = (i, side, q) over the faces
// of its side: sum_j P_q(xi_j) (cUi p_in + cUo p_out) and likewise with the
// pressure weights; fw: the four weights of each face, from the dof's first
// face.  v(c) reads the solution at box-local cell c.  One fixed order.
template <typename V>
__device__ __forceinline__ void trace_moments(const BoxDesc& d, int side, int q,
                                              const double* __restrict__ fw, V v, double& su,
                                              double& sp) {
  const int len = side <= 1 ? d.oby : d.obx;
  su = 0.0;
  sp = 0.0;
  for (int j0 = 0; j0 < len; j0 += 8) {
    f64x2 w[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u < len ? j0 + u : len - 1;
      w[u][0] = *reinterpret_cast<const f64x2*>(fw + 4 * j);
      w[u][1] = *reinterpret_cast<const f64x2*>(fw + 4 * j + 2);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u;
      if (j < len) {
        int ci, co;
        face_cells(d, side, j, ci, co);
        const double pin = v(ci), pout = v(co);
        const double lw = legendre_face(q, j, len);
        const double U = fmat(w[u][0][1], pout, w[u][0][0] * pin);
        const double P = fmat(w[u][1][1], pout, w[u][1][0] * pin);
        su = fmat(lw, U, su);
        sp = fmat(lw, P, sp);
      }
    }
  }
}

// Source-driven solves of the apply, one lane group per subdomain: the
// oversampled problem on hat-Omega_i (box d) with source r and zero Robin
// data, p = its restriction to Omega_i (the owned cells of d), fused with
// the trace moments of the coarse right-hand side (one lane per coarse dof
// of the subdomain, FP64 sums).  Groups past the last subdomain (live =
// false) run along on the last one and write nothing.
template <typename T, typename S, int NB, int GS>
__device__ __forceinline__ void local_body(
    const Blk blk, const BoxDesc* __restrict__ boxes, int m, int group_bytes, int cp_words,
    const S* __restrict__ dinv, const S* __restrict__ coup, const double* __restrict__ r,
    T* __restrict__ p, int nx, const int* __restrict__ dof_off,
    const int* __restrict__ dof_side, const int* __restrict__ dof_q,
    const int* __restrict__ dof_face0, const double* __restrict__ face_w,
    double* __restrict__ mU, double* __restrict__ mP) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i0 = blk.id * (blockDim.x / GS) + grp;
  const bool live = i0 < m;
  const int i = live ? i0 : m - 1;
  BoxSlot<T, S, NB, GS> L(smem_raw + (long long)grp * group_bytes, cp_words);
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const long long origin = (long long)d.y0 * nx + d.x0;
  stage_box(L.us, r, origin, nx, L.cp, coup + d.coff, bx, by, lane, live);
  zero_slots<T, GS>(L.vv, vec_words<NB, GS>(), lane);
  wave_sync();
  if (live && d.pin && lane == 0) L.us[0] = T(0);
  wave_sync();
  // rows from the one across Omega_i's south side (its traces) upward
  box_solve<T, S, NB, GS>(L.us, L.vv, L.cp, dinv + d.doff, bx, by, d.bs, lane,
                         (threadIdx.x & 63) - lane, live, d.oy > 0 ? d.oy - 1 : 0);
  wave_sync();
  if (live && lane >= d.ox && lane < d.ox + d.obx) {
    const long long o2 = origin + (long long)d.oy * nx;
    for (int j = 0; j < d.oby; ++j) p[o2 + (long long)j * nx + lane] = L.us[(d.oy + j) * bx + lane];
  }
  if (!live) return;
  for (int k = dof_off[i] + lane; k < dof_off[i + 1]; k += GS) {
    double su, sp;
    trace_moments(d, dof_side[k], dof_q[k], face_w + 4LL * dof_face0[k],
                  [&](int c) { return (double)L.us[c]; }, su, sp);
    mU[k] = su;
    mP[k] = sp;
  }
}
template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_local(const BoxDesc* __restrict__ boxes, int m, int group_bytes, int cp_words,
            const S* __restrict__ dinv, const S* __restrict__ coup,
            const double* __restrict__ r, T* __restrict__ p, int nx,
            const int* __restrict__ dof_off, const int* __restrict__ dof_side,
            const int* __restrict__ dof_q, const int* __restrict__ dof_face0,
            const double* __restrict__ face_w, double* __restrict__ mU,
            double* __restrict__ mP) {
  local_body<T, S, NB, GS>(hw_blk(), boxes, m, group_bytes, cp_words, dinv, coup, r, p, nx,
                           dof_off, dof_side, dof_q, dof_face0, face_w, mU, mP);
}

// Interface right-hand side in tree order: for tree position t, gsrc[t] =
// {L, R, kind}: kind 0 a flux row, g = -(mU[L] + mU[R]); 1 a pressure row,
// g = -(mP[L] - mP[R]); 2 the replaced row of an all-no-flow grid, g = 0;
// times the row's equilibration scale gscale[t].
__device__ __forceinline__ void coarse_rhs_body(const Blk blk, const int4* __restrict__ gsrc,
                                                const double* __restrict__ gscale,
                                                const double* __restrict__ mU,
                                                const double* __restrict__ mP,
                                                double* __restrict__ g_nd, int np) {
  const int t = blk.id * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int4 src = gsrc[t];
  const double v = src.z == 0 ? -(mU[src.x] + mU[src.y]) : -(mP[src.x] - mP[src.y]);
  g_nd[t] = src.z == 2 ? 0.0 : gscale[t] * v;
}
__global__ void k_coarse_rhs(const int4* __restrict__ gsrc, const double* __restrict__ gscale,
                             const double* __restrict__ mU, const double* __restrict__ mP,
                             double* __restrict__ g_nd, int np) {
  coarse_rhs_body(hw_blk(), gsrc, gscale, mU, mP, g_nd, np);
}

// Refinement residual of the interface solve in tree order: r_nd[t] = g_nd[t]
// - sum over the scaled row of position t of v * x (CSR rp / ci / v), one
// thread per row, terms in row order; blockIdx.y selects a column of a
// multi-column solve (vectors of column k at k * np / k * nc).
__device__ __forceinline__ void coarse_resid_body(const Blk blk, int col,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ g_nd,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ r_nd, int np, int nc) {
  const int t = blk.id * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const double* xk = x + (long long)col * nc;
  double s = g_nd[(long long)col * np + t];
  for (int q = rp[t]; q < rp[t + 1]; ++q) s = fmat(-v[q], xk[ci[q]], s);
  r_nd[(long long)col * np + t] = s;
}
__global__ void k_coarse_resid(const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ v, const double* __restrict__ g_nd,
                               const double* __restrict__ x, double* __restrict__ r_nd, int np,
                               int nc) {
  coarse_resid_body(hw_blk(), blockIdx.y, rp, ci, v, g_nd, x, r_nd, np, nc);
}

// x += dx over n values (columns of a multi-column solve are consecutive).
__device__ __forceinline__ void coarse_add_body(const Blk blk, double* __restrict__ x,
                                                const double* __restrict__ dx, long long n) {
  const long long q = blk.id * (long long)blockDim.x + threadIdx.x;
  if (q < n) x[q] += dx[q];
}
__global__ void k_coarse_add(double* __restrict__ x, const double* __restrict__ dx, long long n) {
  coarse_add_body(hw_blk(), x, dx, n);
}

// ---- interface solve (level-scheduled nested dissection) -------------------
// One launch per tree level and direction; a workgroup takes one chunk, rows
// [row0, row1) of one node's matrix (see device.h).  Each wave takes groups
// of four rows (wave w: rows row0 + 4 w + 16 k); lanes stride the columns
// eight deep, so a wave has 32 matrix loads in flight.  The first group's
// loads are issued before the right-hand side is gathered, so their latency
// overlaps the gather (except at the root of a large tree, whose long gather
// goes first).

// Entries of a node's vector a thread gathers into LDS at a time: a root
// separator of more than kWideRoot rows (kGatherA), a backward border (up to
// kGatherB, as its length needs).
constexpr int kGatherA = 4;
constexpr int kGatherB = 8;
constexpr int kWideRoot = 1024;

// Issue the loads of one 4 x (8 x 64) tile: rows r .. r + 3 (clipped at
// row1), columns b0 + 64 q (clipped at ncol); missing entries read as zero.
__device__ __forceinline__ void load_tile(double (&m)[4][8], const double* __restrict__ M,
                                          int ncol, int r, int row1, int b0) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int b = b0 + 64 * q;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      m[u][q] = (b < ncol && r + u < row1) ? M[(long long)(r + u) * ncol + b] : 0.0;
  }
}

// s[u] += sum_q m[u][q] vec[b0 + 64 q] (vector in LDS).
__device__ __forceinline__ void fma_tile(double (&s)[4], const double (&m)[4][8],
                                         const double* vec, int ncol, int b0) {
  double x[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) x[q] = b0 + 64 * q < ncol ? vec[b0 + 64 * q] : 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] = fmat(m[u][q], x[q], s[u]);
}

// Rows [row0, row1) of M (row-major, ncol columns) times the LDS vector; the
// tile m holds this wave's first tile (rows row0 + 4 wid, columns lane ..),
// and pre(row0 + 4 wid) has already been called.  For every later group of
// four rows r .. r + 3, pre(r) is called first (lane u may fetch what it
// needs for row r + u); then emit(r + u, value) runs in lane u.
template <typename Pre, typename Emit>
__device__ __forceinline__ void gemv_chunk(const double* __restrict__ M, int ncol, int row0,
                                           int row1, const double* vec, double (&m)[4][8],
                                           Pre pre, Emit emit) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = row0 + 4 * wid; r < row1; r += 4 * nw) {
    const bool first = r == row0 + 4 * wid;
    if (!first) pre(r);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    fma_tile(s, m, vec, ncol, lane);
    for (int b0 = lane + 64 * 8; b0 < ncol; b0 += 64 * 8) {
      load_tile(m, M, ncol, r, row1, b0);
      fma_tile(s, m, vec, ncol, b0);
    }
    if (r + 4 * nw < row1) load_tile(m, M, ncol, r + 4 * nw, row1, lane);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double t = wave_sum(s[u]);
      if (lane == u && r + u < row1) emit(r + u, t);
    }
  }
}

// Sums of N values (a power of two, 2..64) over the 64 lanes of the wave, all
// at once: at the exchange with lane ^ off (off = 32, 16, ..., 1) a lane
// keeps half of its values, and the sum of each kept value is its own plus
// the partner's, so every value meets the pairs of wave_sum in the same order
// (each result is bit-identical to wave_sum of that value) with 2N - 1 + 6 -
// log2 N exchanges instead of 6 N.  Afterwards v[0] in lane l is the sum of
// value butterfly_index<N>(l).
template <int N>
__device__ __forceinline__ int butterfly_index(int lane) {
  int idx = 0, n = N;
#pragma unroll
  for (int off = 32; off > 0 && n > 1; off >>= 1) {
    n >>= 1;
    if (lane & off) idx += n;
  }
  return idx;
}
template <int N>
__device__ __forceinline__ void butterfly_sum(double (&v)[N], int lane) {
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int off = 32 >> st;
    const int n = N >> st;  // values still held (compile-time after unrolling)
    if (n > 1) {
      const int half = n >> 1;
      const bool upper = (lane & off) != 0;
#pragma unroll
      for (int i = 0; i < N / 2; ++i)
        if (i < half) {
          const double send = upper ? v[i] : v[i + half];
          const double keep = upper ? v[i + half] : v[i];
          v[i] = keep + __shfl_xor(send, off, 64);
        }
    } else {
      v[0] += __shfl_xor(v[0], off, 64);
    }
  }
}

// A chunk of at most 16 rows and ncol <= 128 columns taken whole by one
// wave: lane l loads columns l and l + 64 of every row, all at once, and the
// sixteen row sums are reduced together; afterwards lane l holds the sum of
// row row0 + butterfly_index<16>(l).  Each lane's partial sums and the
// reduction tree are those of gemv_chunk, so the results are the same.
__device__ __forceinline__ void load_chunk16(double (&m)[16][2], const double* __restrict__ M,
                                             int ncol, int row0, int row1, int lane) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int b = lane + 64 * q;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      m[u][q] = (b < ncol && row0 + u < row1) ? M[(long long)(row0 + u) * ncol + b] : 0.0;
  }
}
__device__ __forceinline__ double gemv_chunk16(const double (&m)[16][2], const double* vec,
                                               int ncol, int lane) {
  double x[2], s[16];
#pragma unroll
  for (int q = 0; q < 2; ++q) x[q] = lane + 64 * q < ncol ? vec[lane + 64 * q] : 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s[u] = 0.0;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int u = 0; u < 16; ++u) s[u] = fmat(m[u][q], x[q], s[u]);
  butterfly_sum<16>(s, lane);
  return s[0];
}
// Whether a forward chunk is taken whole, 16 rows per wave (wave w: rows
// row0 + 16 w .. row0 + 16 w + 15) with every row's columns in the wave's
// registers.
__device__ __forceinline__ bool whole_chunk(const CChunk& ch, int ncol) {
  return ncol <= 128 && ch.row1 - ch.row0 <= 16 * (int)(blockDim.x >> 6);
}
// Whether a backward chunk is taken whole by a one-wave workgroup.
__device__ __forceinline__ bool whole_chunk_wave(const CChunk& ch, int ncol) {
  return blockDim.x == 64 && ncol <= 128 && ch.row1 - ch.row0 <= 16;
}

// Forward level: for the separator rows a of the chunk's node (tree
// positions t = yoff + a),
//   v[a] = g_nd[t] - (contributions of the descendants, in slot order),
// with the contributions by destination in contrib[u * np + t] (slot u,
// zero where unused).  Then rows of [W; E] v: y_F into ybuf (straight into
// x through idx for a node without border rows, whose x_F = y_F), each c_n
// row into its destination slot cdest[coff + row - nf].
__device__ __forceinline__ void coarse_fwd_body(
    const CChunk ch, const double* __restrict__ fwd, const double* __restrict__ g_nd,
    double* __restrict__ contrib, int maxp, int np, const int* __restrict__ cdest,
    double* __restrict__ ybuf, const int* __restrict__ idx, double* __restrict__ x) {
  extern __shared__ double v[];
  const int nf = ch.nf, lane = threadIdx.x & 63;
  const double* M = fwd + ch.mat;
  const int yoff = ch.yoff, coff = ch.coff;
  int dst = -1;
  // v[a] = g_nd[t] minus the contributions in slot order; a thread takes
  // its entries A at a time, with all their loads in flight together
  auto gather_rows = [&](auto A) {
    constexpr int kA = decltype(A)::value, kC = kA > 1 ? 4 : 8;
    const int bd = blockDim.x;
    for (int a0 = threadIdx.x; a0 < nf; a0 += kA * bd) {
      long long t[kA];
      double s[kA];
#pragma unroll
      for (int i = 0; i < kA; ++i) {
        const int a = a0 + i * bd;
        t[i] = (long long)yoff + (a < nf ? a : nf - 1);
        s[i] = g_nd[t[i]];
      }
      for (int u0 = 0; u0 < maxp; u0 += kC) {
        double c[kA][kC];
#pragma unroll
        for (int i = 0; i < kA; ++i)
#pragma unroll
          for (int k = 0; k < kC; ++k)
            c[i][k] = u0 + k < maxp ? contrib[(long long)(u0 + k) * np + t[i]] : 0.0;
#pragma unroll
        for (int i = 0; i < kA; ++i)
#pragma unroll
          for (int k = 0; k < kC; ++k)
            if (u0 + k < maxp) s[i] -= c[i][k];
      }
#pragma unroll
      for (int i = 0; i < kA; ++i)
        if (a0 + i * bd < nf) v[a0 + i * bd] = s[i];
    }
    __syncthreads();
  };
  auto gather = [&]() { gather_rows(std::integral_constant<int, 1>()); };
  auto emit = [&](int row, double val) {
    if (row >= nf)
      contrib[dst] = val;
    else if (ch.nu == 0)
      x[idx[ch.fcol + row]] = val;  // a node without border rows: x_F = y_F
    else
      ybuf[yoff + row] = val;
  };
  if (whole_chunk(ch, nf)) {
    const int r0 = ch.row0 + 16 * (int)(threadIdx.x >> 6);
    double m[16][2];
    load_chunk16(m, M, nf, r0, ch.row1, lane);
    const int row = r0 + butterfly_index<16>(lane);
    dst = (row >= nf && row < ch.row1) ? cdest[coff + row - nf] : -1;
    gather();
    const double val = gemv_chunk16(m, v, nf, lane);
    if ((lane & 3) == 0 && row < ch.row1) emit(row, val);
    return;
  }
  auto pre = [&](int r) {
    const int row = r + lane;
    dst = (lane < 4 && row >= nf && row < ch.row1) ? cdest[coff + row - nf] : -1;
  };
  double m[4][8];
  const int rw = ch.row0 + 4 * (threadIdx.x >> 6);
  if (ch.nu == 0 && nf > kWideRoot) {
    // the root of a large tree: few workgroups, each with a long gather,
    // which goes first, kGatherA entries deep (the tile's registers are
    // not live yet, so the kernel's occupancy holds)
    gather_rows(std::integral_constant<int, kGatherA>());
    load_tile(m, M, nf, rw, ch.row1, lane);
    pre(rw);
  } else {
    load_tile(m, M, nf, rw, ch.row1, lane);
    pre(rw);
    gather();
  }
  gemv_chunk(M, nf, ch.row0, ch.row1, v, m, pre, emit);
}
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_fwd(const CChunk* __restrict__ chunks, const double* __restrict__ fwd,
                 const double* __restrict__ g_nd, double* __restrict__ contrib, int maxp, int np,
                 const int* __restrict__ cdest, double* __restrict__ ybuf,
                 const int* __restrict__ idx, double* __restrict__ x) {
  coarse_fwd_body(chunks[blockIdx.x], fwd, g_nd, contrib, maxp, np, cdest, ybuf, idx, x);
}

// Backward level: x_F = y_F - G x_U for the chunk's rows (x_U gathered
// through idx[ucol ..], x_F scattered through idx[fcol ..]; nu > 0).
__device__ __forceinline__ void coarse_bwd_body(const CChunk ch, const double* __restrict__ bwd,
                                                const int* __restrict__ idx,
                                                const double* __restrict__ ybuf,
                                                double* __restrict__ x) {
  extern __shared__ double xu[];
  const int nu = ch.nu, lane = threadIdx.x & 63;
  const double* M = bwd + ch.mat;
  const int yoff = ch.yoff, fcol = ch.fcol;
  int dst = 0;
  double y = 0.0;
  // xu[b] = x[idx[ucol + b]]: a thread takes its entries R at a time, all
  // their loads in flight together, R being 1, 2, 4 or kGatherB as the
  // border needs (it is the same in the whole workgroup)
  auto gather_r = [&](auto R) {
    constexpr int kR = decltype(R)::value;
    const int bd = blockDim.x;
    for (int b0 = threadIdx.x; b0 < nu; b0 += kR * bd) {
      int k[kR];
      double val[kR];
#pragma unroll
      for (int i = 0; i < kR; ++i) {
        const int b = b0 + i * bd;
        k[i] = idx[ch.ucol + (b < nu ? b : nu - 1)];
      }
#pragma unroll
      for (int i = 0; i < kR; ++i) val[i] = x[k[i]];
#pragma unroll
      for (int i = 0; i < kR; ++i)
        if (b0 + i * bd < nu) xu[b0 + i * bd] = val[i];
    }
    __syncthreads();
  };
  auto gather = [&]() {
    const int rounds = (nu + (int)blockDim.x - 1) / (int)blockDim.x;
    if (rounds <= 1)
      gather_r(std::integral_constant<int, 1>());
    else if (rounds <= 2)
      gather_r(std::integral_constant<int, 2>());
    else if (rounds <= 4)
      gather_r(std::integral_constant<int, 4>());
    else
      gather_r(std::integral_constant<int, kGatherB>());
  };
  if (whole_chunk_wave(ch, nu)) {
    double m[16][2];
    load_chunk16(m, M, nu, ch.row0, ch.row1, lane);
    const int row = ch.row0 + butterfly_index<16>(lane);
    if (row < ch.row1) {
      dst = idx[fcol + row];
      y = ybuf[yoff + row];
    }
    gather();
    const double val = gemv_chunk16(m, xu, nu, lane);
    if ((lane & 3) == 0 && row < ch.row1) x[dst] = y - val;
    return;
  }
  auto pre = [&](int r) {
    const int row = r + lane;
    if (lane < 4 && row < ch.row1) {
      dst = idx[fcol + row];
      y = ybuf[yoff + row];
    }
  };
  double m[4][8];
  const int rw = ch.row0 + 4 * (threadIdx.x >> 6);
  load_tile(m, M, nu, rw, ch.row1, lane);
  pre(rw);
  gather();
  gemv_chunk(M, nu, ch.row0, ch.row1, xu, m, pre, [&](int, double val) { x[dst] = y - val; });
}
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_bwd(const CChunk* __restrict__ chunks, const double* __restrict__ bwd,
                 const int* __restrict__ idx, const double* __restrict__ ybuf,
                 double* __restrict__ x) {
  coarse_bwd_body(chunks[blockIdx.x], bwd, idx, ybuf, x);
}

// p[Omega_i] += P_i x_i (multiscale reconstruction; Omega_i is the owned part
// of box d), one workgroup per subdomain.
template <typename T, typename S>
__device__ __forceinline__ void reconstruct_body(const Blk blk, const BoxDesc* __restrict__ boxes,
                                                 const S* __restrict__ mbf,
                                                 const long long* __restrict__ mbf_off,
                                                 const int* __restrict__ dof_off,
                                                 const double* __restrict__ xc,
                                                 T* __restrict__ p, int nx) {
  __shared__ T xs[64];
  const int i = blk.id;
  const BoxDesc d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0, ncell = d.obx * d.oby;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) xs[k] = (T)xc[k0 + k];
  __syncthreads();
  const S* P = mbf + mbf_off[i];
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % d.obx, j = q / d.obx;
    const long long c = (long long)(d.y0 + d.oy + j) * nx + d.x0 + d.ox + a;
    T s = p[c];
    for (int k = 0; k < nk; ++k) s = fmat((T)P[(long long)k * ncell + q], xs[k], s);
    p[c] = s;
  }
}
template <typename T, typename S>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct(const BoxDesc* __restrict__ boxes, const S* __restrict__ mbf,
                  const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                  const double* __restrict__ xc, T* __restrict__ p, int nx) {
  reconstruct_body<T, S>(hw_blk(), boxes, mbf, mbf_off, dof_off, xc, p, nx);
}

// Smoothing residual rho = r - A p.
template <typename T>
__device__ __forceinline__ void residual_body(const Blk blk, const T* __restrict__ tx,
                                              const T* __restrict__ ty, int nx, int ny,
                                              const double* __restrict__ r,
                                              const T* __restrict__ p, T* __restrict__ rho) {
  const long long n = (long long)nx * ny;
  for (long long c = blk.id * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)blk.n * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    rho[c] = (T)r[c] - stencil(tx, ty, nx, ny, ix, iy, p);
  }
}
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_residual(const T* __restrict__ tx, const T* __restrict__ ty, int nx, int ny,
               const double* __restrict__ r, const T* __restrict__ p, T* __restrict__ rho) {
  residual_body<T>(hw_blk(), tx, ty, nx, ny, r, p, rho);
}

// Restricted additive Schwarz: solve A[S_i] e = rho[S_i] on patch i (one
// lane group per patch) and add e on the owned subdomain Omega_i (each cell
// is written by one patch only).  Groups past the last patch run along on
// the last one and write nothing.
template <typename T, typename S, int NB, int GS>
__device__ __forceinline__ void patch_body(const Blk blk, const BoxDesc* __restrict__ boxes,
                                           int m, int group_bytes, int cp_words,
                                           const S* __restrict__ dinv,
                                           const S* __restrict__ coup,
                                           const T* __restrict__ rho, T* __restrict__ p,
                                           int nx) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i0 = blk.id * (blockDim.x / GS) + grp;
  const bool live = i0 < m;
  const int i = live ? i0 : m - 1;
  BoxSlot<T, S, NB, GS> L(smem_raw + (long long)grp * group_bytes, cp_words);
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const long long origin = (long long)d.y0 * nx + d.x0;
  stage_box(L.us, rho, origin, nx, L.cp, coup + d.coff, bx, by, lane, live);
  zero_slots<T, GS>(L.vv, vec_words<NB, GS>(), lane);
  wave_sync();
  if (live && d.pin && lane == 0) L.us[0] = T(0);
  wave_sync();
  // the owned rows upward
  box_solve<T, S, NB, GS>(L.us, L.vv, L.cp, dinv + d.doff, bx, by, d.bs, lane,
                         (threadIdx.x & 63) - lane, live, d.oy);
  wave_sync();
  // p += e on the owned cells, sixteen rows of read-modify-write in flight
  const bool own = live && lane >= d.ox && lane < d.ox + d.obx;
  const int col = own ? lane : d.ox;
  const long long o2 = origin + (long long)d.oy * nx;
  const int rows = wave_max(live ? d.oby : 0);
  for (int j0 = 0; j0 < rows; j0 += 16) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + u < d.oby ? j0 + u : d.oby - 1;
      v[u] = p[o2 + (long long)j * nx + col];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (own && j0 + u < d.oby)
        p[o2 + (long long)(j0 + u) * nx + lane] = v[u] + L.us[(d.oy + j0 + u) * bx + lane];
  }
}
template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_patch(const BoxDesc* __restrict__ boxes, int m, int group_bytes, int cp_words,
            const S* __restrict__ dinv, const S* __restrict__ coup, const T* __restrict__ rho,
            T* __restrict__ p, int nx) {
  patch_body<T, S, NB, GS>(hw_blk(), boxes, m, group_bytes, cp_words, dinv, coup, rho, p, nx);
}

template <typename T>
__device__ __forceinline__ void sum_body(const Blk blk, const T* __restrict__ p, long long n,
                                         double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long st = (long long)blk.n * blockDim.x;
  double s = 0.0;
  for (long long c0 = blk.id * (long long)blockDim.x + threadIdx.x; c0 < n;
       c0 += kRound * st) {
    T a[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = p[c < n ? c : n - 1];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
      if (c0 + u * st < n) s += (double)a[u];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blk.id] = s;
}
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_sum(const T* __restrict__ p, long long n, double* __restrict__ partials) {
  sum_body<T>(hw_blk(), p, n, partials);
}

// z = p - mean(p) (no-flow) or z = p, in FP64.  First round loaded before
// the reduction, as in k_mgs_step.
template <typename T>
__device__ __forceinline__ void finalize_body(const Blk blk, const T* __restrict__ p, long long n,
                                              const double* __restrict__ partials, int nb,
                                              double* __restrict__ z) {
  __shared__ double red[kVecThreads / 64];
  const long long st = (long long)blk.n * blockDim.x;
  T a[kRound];
  auto load = [&](long long c0) {
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = p[c < n ? c : n - 1];
    }
  };
  const long long start = blk.id * (long long)blockDim.x + threadIdx.x;
  load(start);
  const double mean = partials ? reduce_partials(partials, nb, red) / (double)n : 0.0;
  for (long long c0 = start; c0 < n; c0 += kRound * st) {
    if (c0 != start) load(c0);
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) z[c] = (double)a[u] - mean;
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_finalize(const T* __restrict__ p, long long n, const double* __restrict__ partials, int nb,
               double* __restrict__ z) {
  finalize_body<T>(hw_blk(), p, n, partials, nb, z);
}

__global__ void k_convert(const double* __restrict__ s, float* __restrict__ d, long long n) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    d[c] = (float)s[c];
}

// ---- GMRES -----------------------------------------------------------------
// (Grid-stride loops in rounds of kRound elements, see reduce_partials.)

// r = b - A p (b when p is null), partial sums of r^2.
__global__ void __launch_bounds__(kVecThreads)
    k_resid_norm(const double* __restrict__ tx, const double* __restrict__ ty, int nx, int ny,
                 const double* __restrict__ b, const double* __restrict__ p,
                 double* __restrict__ r, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long n = (long long)nx * ny, st = (long long)gridDim.x * blockDim.x;
  double s = 0.0;
  for (long long c0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; c0 < n;
       c0 += kRound * st) {
    double v[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st, q = c < n ? c : n - 1;
      const int iy = (int)(q / nx), ix = (int)(q - (long long)iy * nx);
      v[u] = p ? b[q] - stencil(tx, ty, nx, ny, ix, iy, p) : b[q];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) {
        r[c] = v[u];
        s += v[u] * v[u];
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_zero(double* __restrict__ v, long long n) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    v[c] = 0.0;
}

__global__ void k_scale(double* __restrict__ v, long long n, double alpha) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    v[c] *= alpha;
}

// w = A z, partial sums of w . v0.
__device__ __forceinline__ void arnoldi_start_body(const Blk blk, const double* __restrict__ tx,
                                                   const double* __restrict__ ty, int nx, int ny,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ w,
                                                   const double* __restrict__ v0,
                                                   double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long n = (long long)nx * ny, st = (long long)blk.n * blockDim.x;
  double s = 0.0;
  for (long long c0 = blk.id * (long long)blockDim.x + threadIdx.x; c0 < n;
       c0 += kRound * st) {
    double v[kRound], o[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st, q = c < n ? c : n - 1;
      const int iy = (int)(q / nx), ix = (int)(q - (long long)iy * nx);
      v[u] = stencil(tx, ty, nx, ny, ix, iy, z);
      o[u] = v0[q];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) {
        w[c] = v[u];
        s += v[u] * o[u];
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blk.id] = s;
}
__global__ void __launch_bounds__(kVecThreads)
    k_arnoldi_start(const double* __restrict__ tx, const double* __restrict__ ty, int nx, int ny,
                    const double* __restrict__ z, double* __restrict__ w,
                    const double* __restrict__ v0, double* __restrict__ partials) {
  arnoldi_start_body(hw_blk(), tx, ty, nx, ny, z, w, v0, partials);
}

// h = sum(part_in) (= w . v_i); hcol[i] = h; w -= h v_i; partial sums of
// w . v_next, or of w . w when vnext is null.  The vectors' loads do not
// depend on h: every thread issues its first round before the reduction
// that forms h (outside any loop, so its barriers are met by all threads),
// then finishes its remaining rounds.
__device__ __forceinline__ void mgs_step_body(const Blk blk, const double* __restrict__ part_in,
                                              double* __restrict__ part_out, int nb,
                                              double* __restrict__ hcol, int i,
                                              double* __restrict__ w,
                                              const double* __restrict__ vi,
                                              const double* __restrict__ vnext, long long n) {
  __shared__ double red[kVecThreads / 64];
  const bool self = vnext == nullptr;
  const double* vn = self ? vi : vnext;
  const long long st = (long long)blk.n * blockDim.x;
  double a[kRound], b[kRound], d[kRound];
  auto load = [&](long long c0) {
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st, q = c < n ? c : n - 1;
      a[u] = w[q];
      b[u] = vi[q];
      d[u] = vn[q];
    }
  };
  double s = 0.0, h = 0.0;
  auto use = [&](long long c0) {
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) {
        const double v = a[u] - h * b[u];
        w[c] = v;
        s += v * (self ? v : d[u]);
      }
    }
  };
  const long long start = blk.id * (long long)blockDim.x + threadIdx.x;
  load(start);
  h = reduce_partials(part_in, nb, red);
  if (blk.id == 0 && threadIdx.x == 0) hcol[i] = h;
  use(start);
  for (long long c0 = start + kRound * st; c0 < n; c0 += kRound * st) {
    load(c0);
    use(c0);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part_out[blk.id] = s;
}
__global__ void __launch_bounds__(kVecThreads)
    k_mgs_step(const double* __restrict__ part_in, double* __restrict__ part_out, int nb,
               double* __restrict__ hcol, int i, double* __restrict__ w,
               const double* __restrict__ vi, const double* __restrict__ vnext, long long n) {
  mgs_step_body(hw_blk(), part_in, part_out, nb, hcol, i, w, vi, vnext, n);
}

// hn = sqrt(sum(part_in)); hcol[j] = hn; w /= hn (if hn > 0).  First round
// loaded before the reduction, as in k_mgs_step.
__device__ __forceinline__ void norm_scale_body(const Blk blk, const double* __restrict__ part_in,
                                                int nb, double* __restrict__ hcol, int j,
                                                double* __restrict__ w, long long n) {
  __shared__ double red[kVecThreads / 64];
  const long long st = (long long)blk.n * blockDim.x;
  double a[kRound];
  auto load = [&](long long c0) {
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = w[c < n ? c : n - 1];
    }
  };
  const long long start = blk.id * (long long)blockDim.x + threadIdx.x;
  load(start);
  const double hn = sqrt(reduce_partials(part_in, nb, red));
  if (blk.id == 0 && threadIdx.x == 0) hcol[j] = hn;
  if (!(hn > 0.0)) return;
  const double inv = 1.0 / hn;
  for (long long c0 = start; c0 < n; c0 += kRound * st) {
    if (c0 != start) load(c0);
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) w[c] = a[u] * inv;
    }
  }
}
__global__ void __launch_bounds__(kVecThreads)
    k_norm_scale(const double* __restrict__ part_in, int nb, double* __restrict__ hcol, int j,
                 double* __restrict__ w, long long n) {
  norm_scale_body(hw_blk(), part_in, nb, hcol, j, w, n);
}

// p += sum_{i < k} y_i Z_i (k <= kMaxUpdate per launch).
constexpr int kMaxUpdate = 16;
__global__ void k_update(double* __restrict__ p, const double* __restrict__ Z,
                         const double* __restrict__ y, int k, long long n) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    double z[kMaxUpdate];
#pragma unroll
    for (int i = 0; i < kMaxUpdate; ++i) z[i] = Z[(long long)(i < k ? i : 0) * n + c];
    double s = p[c];
#pragma unroll
    for (int i = 0; i < kMaxUpdate; ++i)
      if (i < k) s += y[i] * z[i];
    p[c] = s;
  }
}

// partial sums of x^2.
__global__ void __launch_bounds__(kVecThreads)
    k_sumsq(const double* __restrict__ x, long long n, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const long long st = (long long)gridDim.x * blockDim.x;
  double s = 0.0;
  for (long long c0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; c0 < n;
       c0 += kRound * st) {
    double a[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = x[c < n ? c : n - 1];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
      if (c0 + u * st < n) s += a[u] * a[u];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ---- several right-hand sides per launch ----------------------------------
// The kernels below apply T to K <= kMaxRhs right-hand sides at once (vectors
// given by per-RHS base pointers).  Every per-RHS sum runs in the order of
// the one-RHS kernels above, so the results are those of K separate
// applications, bit for bit; what the K columns share is each load of a
// factor quad, an MBF entry or an interface-matrix tile, and each step of
// the row recurrence of a box.

template <typename T>
struct RhsPtrs {
  T* v[kMaxRhs];
};

// Blocks in flight per lane for K right-hand sides: about 64 VGPRs of rows
// (the K columns need their own registers), 2 or 4.
template <typename S, int NB, int K>
constexpr int reg_depth_k() {
  constexpr int per_block = half_rows(NB) * (int)sizeof(S) / 4;
  constexpr int d = pow2_depth((K == 1 ? 96 : 64) / per_block);
  return d > 4 ? 4 : d;
}

// acc[k] = sum_c D(rc, c) v_k[c] for the K vectors of the group (column k's
// doubled copy at vo / vr + k * VW): each factor entry is converted once and
// used for every column; per column, the order of half_dot.  A scheduling
// barrier after each group of four entries keeps the compiler from hoisting
// all the vector reads at once (which would need more registers than a lane
// has).
template <typename T, typename S, int NB, int K, int VW>
__device__ __forceinline__ void half_dot_k(const HalfRow<S, NB>& d, const S (&rot)[Half<NB>::H],
                                           const T* vo, const T* vr, T (&acc)[K]) {
  constexpr int NH = Half<NB>::NH, K0 = Half<NB>::K0, H = Half<NB>::H;
  T a[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k) a[k][0] = a[k][1] = a[k][2] = a[k][3] = T(0);
#pragma unroll
  for (int q = 0; q < NH; ++q) {
    const T dq[4] = {(T)d.q[q][0], (T)d.q[q][1], (T)d.q[q][2], (T)d.q[q][3]};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) a[k][i] = fmat(dq[i], vo[k * VW + K0 + 4 * q + i], a[k][i]);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int e = 0; e < K0; ++e) {
    const T de = (T)d.h[e];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k][e] = fmat(de, vo[k * VW + e], a[k][e]);
  }
#pragma unroll
  for (int g = 1; g <= H; g += 4) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = g; e < g + 4 && e <= H; ++e) {
      const T de = (T)rot[e - 1];
#pragma unroll
      for (int k = 0; k < K; ++k)
        a[k][(e - 1) & 3] = fmat(de, vr[k * VW - e], a[k][(e - 1) & 3]);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = (a[k][0] + a[k][1]) + (a[k][2] + a[k][3]);
}

// Completes this work-item's global stores before its later loads and makes
// them visible to the group (workgroup scope: waits only, no cache flush).
__device__ __forceinline__ void group_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Block LDL^T solves of one box for K right-hand sides by a group (the
// recurrence of box_solve, K columns per step).  Row j of right-hand side k
// is read at in[k] + j * istride (lane r: column r); the solution is built
// in place at work[k] + j * wstride: the forward pass leaves u_j there and
// the backward pass overwrites it with x_j.  The next step's rows are loaded
// one step ahead.  vv holds the group's K vector slots (vec_words each,
// zeroed), cp the couplings (LDS); g0 is the group's first lane in the wave;
// pin zeroes b_0 in column 0 (a box fixed at its first cell); the backward
// pass ends at row stop, as in box_solve.
template <typename T, typename S, int NB, int GS, int K, typename In>
__device__ __forceinline__ void box_solve_k(const In* const (&in)[K], long long istride,
                                            T* const (&work)[K], long long wstride, T* vv,
                                            const S* cp, const S* __restrict__ Dinv, int bx,
                                            int by, int bstride, int r, int g0, bool live,
                                            bool pin, int stop) {
  constexpr int H = Half<NB>::H, VW = vec_words<NB, GS>();
  constexpr int DEPTH = reg_depth_k<S, NB, K>();
  const bool act = live && r < bx;
  const int rc = r < bx ? r : bx - 1;
  int src[(H + 3) / 4];
  mirror_lanes<H>(src, g0, rc, bx);
  const T* vo = vv + H + rc;
  const T* vr = vv + H + rc + bx;
  T carry[K], nxt[K];
#pragma unroll
  for (int k = 0; k < K; ++k) carry[k] = T(0);
  auto in_row = [&](int s) {
    const long long off = (long long)(s < by ? s : by - 1) * istride + rc;
#pragma unroll
    for (int k = 0; k < K; ++k) nxt[k] = (T)in[k][off];
  };
  in_row(0);
  pipelined_sweep<S, NB, DEPTH>(
      live ? by : 0, wave_steps<DEPTH>(live ? by : 0), [](int s) { return s; },
      [&](int s, const HalfRow<S, NB>& d, bool valid) {
        S rot[H];
        mirror_rows<S, NB>(rot, d, src);
        const int j = s < by ? s : by - 1;
        const bool w = act && valid;
        T b[K];
#pragma unroll
        for (int k = 0; k < K; ++k) b[k] = (pin && j == 0 && rc == 0) ? T(0) : nxt[k];
        in_row(s + 1);
        const T cj = (T)cp[j * bx + rc];
        if (r < bx)
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const T y = j > 0 ? fmat(cj, carry[k], b[k]) : b[k];
            vv[k * VW + H + r] = vv[k * VW + H + bx + r] = w ? y : T(0);
          }
        wave_sync();
        T acc[K];
        half_dot_k<T, S, NB, K, VW>(d, rot, vo, vr, acc);
        wave_sync();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (w) work[k][(long long)j * wstride + r] = acc[k];
          carry[k] = w ? acc[k] : carry[k];
        }
      },
      Dinv, bstride, bx, rc);
  group_fence();
  // carry = x_{by-1} = u_{by-1}; rows by - 2 down to stop
  const int nb = live && by - 1 - stop > 0 ? by - 1 - stop : 0;
  auto u_row = [&](int s) {
    int j = by - 2 - s;
    j = j < 0 ? 0 : j;
#pragma unroll
    for (int k = 0; k < K; ++k) nxt[k] = work[k][(long long)j * wstride + rc];
  };
  u_row(0);
  pipelined_sweep<S, NB, DEPTH>(
      nb, wave_steps<DEPTH>(nb), [by](int s) { return by - 2 - s; },
      [&](int s, const HalfRow<S, NB>& d, bool valid) {
        S rot[H];
        mirror_rows<S, NB>(rot, d, src);
        int j = by - 2 - s;
        j = j < 0 ? 0 : j;
        const int jn = j + 1 < by ? j + 1 : by - 1;
        const bool w = act && valid;
        T u[K];
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = nxt[k];
        u_row(s + 1);
        const T cj = (T)cp[jn * bx + rc];
        if (r < bx)
#pragma unroll
          for (int k = 0; k < K; ++k)
            vv[k * VW + H + r] = vv[k * VW + H + bx + r] = w ? cj * carry[k] : T(0);
        wave_sync();
        T acc[K];
        half_dot_k<T, S, NB, K, VW>(d, rot, vo, vr, acc);
        wave_sync();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const T xj = u[k] + acc[k];
          if (w) work[k][(long long)j * wstride + r] = xj;
          carry[k] = w ? xj : carry[k];
        }
      },
      Dinv, bstride, bx, rc);
  group_fence();
}

// LDS slot of one lane group for K right-hand sides:
//   vv[K][vec_words] (T) | cp[max cells] (S).
template <typename T, typename S, int NB, int GS, int K>
struct BoxSlotK {
  T* vv;
  S* cp;
  __device__ BoxSlotK(char* base) {
    vv = reinterpret_cast<T*>(base);
    cp = reinterpret_cast<S*>(base + K * vec_words<NB, GS>() * sizeof(T));
  }
};

// k_local for K right-hand sides: the oversampled solve of every column,
// built in the subdomain's slice of the scratch vectors (offset coff, row
// stride bx), p_k = its restriction to Omega_i, and the trace moments of
// every coarse dof of the subdomain for every k (mU[k * nc + dof], mP
// likewise; the arithmetic of k_local per column).
template <typename T, typename S, int NB, int K, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_local_k(const BoxDesc* __restrict__ boxes, int m, int group_bytes,
              const S* __restrict__ dinv, const S* __restrict__ coup, RhsPtrs<const double> r,
              RhsPtrs<T> p, RhsPtrs<T> e, int nx, const int* __restrict__ dof_off,
              const int* __restrict__ dof_side, const int* __restrict__ dof_q,
              const int* __restrict__ dof_face0, const double* __restrict__ face_w,
              double* __restrict__ mU, double* __restrict__ mP, int nc) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i0 = blockIdx.x * (blockDim.x / GS) + grp;
  const bool live = i0 < m;
  const int i = live ? i0 : m - 1;
  BoxSlotK<T, S, NB, GS, K> L(smem_raw + (long long)grp * group_bytes);
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const long long origin = (long long)d.y0 * nx + d.x0;
  const double* in[K];
  T* work[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    in[k] = r.v[k] + origin;
    work[k] = e.v[k] + d.coff;
  }
  words_to_lds<S, GS>(L.cp, coup + d.coff, bx * by, lane, live);
  zero_slots<T, GS>(L.vv, K * vec_words<NB, GS>(), lane);
  wave_sync();
  box_solve_k<T, S, NB, GS, K, double>(in, nx, work, bx, L.vv, L.cp, dinv + d.doff, bx, by,
                                       d.bs, lane, (threadIdx.x & 63) - lane, live,
                                       live && d.pin, d.oy > 0 ? d.oy - 1 : 0);
  if (!live) return;
  if (lane >= d.ox && lane < d.ox + d.obx) {
    const long long o2 = origin + (long long)d.oy * nx;
#pragma unroll 1
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < d.oby; ++j)
        p.v[k][o2 + (long long)j * nx + lane] = work[k][(long long)(d.oy + j) * bx + lane];
  }
  for (int kd = dof_off[i] + lane; kd < dof_off[i + 1]; kd += GS) {
    const int side = dof_side[kd], q = dof_q[kd];
    const double* fw = face_w + 4LL * dof_face0[kd];
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      const T* wk = work[k];
      double su, sp;
      trace_moments(d, side, q, fw, [&](int c) { return (double)wk[c]; }, su, sp);
      mU[(long long)k * nc + kd] = su;
      mP[(long long)k * nc + kd] = sp;
    }
  }
}

// k_patch for K right-hand sides: e_k = A[S_i]^-1 rho_k[S_i], built in the
// patch's slice of the scratch vectors (offset coff, row stride bx), then
// p_k += e_k on the owned cells.
template <typename T, typename S, int NB, int K, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_patch_k(const BoxDesc* __restrict__ boxes, int m, int group_bytes,
              const S* __restrict__ dinv, const S* __restrict__ coup, RhsPtrs<const T> rho,
              RhsPtrs<T> p, RhsPtrs<T> e, int nx) {
  extern __shared__ __align__(16) char smem_raw[];
  const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int i0 = blockIdx.x * (blockDim.x / GS) + grp;
  const bool live = i0 < m;
  const int i = live ? i0 : m - 1;
  BoxSlotK<T, S, NB, GS, K> L(smem_raw + (long long)grp * group_bytes);
  const BoxDesc d = boxes[i];
  const int bx = d.bx, by = d.by;
  const long long origin = (long long)d.y0 * nx + d.x0;
  const T* in[K];
  T* work[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    in[k] = rho.v[k] + origin;
    work[k] = e.v[k] + d.coff;
  }
  words_to_lds<S, GS>(L.cp, coup + d.coff, bx * by, lane, live);
  zero_slots<T, GS>(L.vv, K * vec_words<NB, GS>(), lane);
  wave_sync();
  box_solve_k<T, S, NB, GS, K, T>(in, nx, work, bx, L.vv, L.cp, dinv + d.doff, bx, by, d.bs,
                                  lane, (threadIdx.x & 63) - lane, live, live && d.pin, d.oy);
  // p += e on the owned cells, eight rows of read-modify-write in flight
  const bool own = live && lane >= d.ox && lane < d.ox + d.obx;
  const int col = own ? lane : d.ox;
  const long long o2 = origin + (long long)d.oy * nx;
  const int rows = wave_max(live ? d.oby : 0);
#pragma unroll 1
  for (int k = 0; k < K; ++k) {
    T* pk = p.v[k];
    const T* ek = work[k] + (long long)d.oy * bx;
    for (int j0 = 0; j0 < rows; j0 += 8) {
      T v[8], ev[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u < d.oby ? j0 + u : d.oby - 1;
        v[u] = pk[o2 + (long long)j * nx + col];
        ev[u] = ek[(long long)j * bx + col];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (own && j0 + u < d.oby) pk[o2 + (long long)(j0 + u) * nx + lane] = v[u] + ev[u];
    }
  }
}

// Interface right-hand sides of K columns (blockIdx.y = column; vectors of
// column k at offset k * nc / k * np).
__global__ void k_coarse_rhs_k(const int4* __restrict__ gsrc, const double* __restrict__ gscale,
                               const double* __restrict__ mU, const double* __restrict__ mP,
                               double* __restrict__ g_nd, int np, int nc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const long long ko = (long long)blockIdx.y * nc;
  const int4 src = gsrc[t];
  const double v = src.z == 0 ? -(mU[ko + src.x] + mU[ko + src.y])
                              : -(mP[ko + src.x] - mP[ko + src.y]);
  g_nd[(long long)blockIdx.y * np + t] = src.z == 2 ? 0.0 : gscale[t] * v;
}

// s[u][k] += sum_q m[u][q] vec_k[b0 + 64 q] for the K columns vec + k * ld
// (LDS): per (u, k) the order of fma_tile.  One column at a time (a
// scheduling barrier after each keeps the LDS reads of later columns from
// being hoisted into registers).
template <int K>
__device__ __forceinline__ void fma_tile_k(double (&s)[4][K], const double (&m)[4][8],
                                           const double* vec, int ld, int ncol, int b0) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = b0 + 64 * q < ncol ? vec[k * ld + b0 + 64 * q] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u][k] = fmat(m[u][q], x[q], s[u][k]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// gemv_chunk for K columns of the LDS matrix vec (column k at vec + k * ld).
// After the butterfly, lane l holds output (row r + u_l, column k_l) with
// u_l * K + k_l = butterfly_index(l); pre(row, k) runs in every lane for its
// own output before that group's tile loads, and emit(row, k, value) in one
// lane per output.
template <int K, typename Pre, typename Emit>
__device__ __forceinline__ void gemv_chunk_k(const double* __restrict__ M, int ncol, int row0,
                                             int row1, const double* vec, int ld,
                                             double (&m)[4][8], Pre pre, Emit emit) {
  constexpr int N = 4 * K;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int bi = butterfly_index<N>(lane);
  const int ul = bi / K, kl = bi % K;
  const bool emitter = (lane & (64 / N - 1)) == 0;
  for (int r = row0 + 4 * wid; r < row1; r += 4 * nw) {
    const bool first = r == row0 + 4 * wid;
    if (!first) pre(r + ul, kl);
    double s[4][K];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) s[u][k] = 0.0;
    fma_tile_k<K>(s, m, vec, ld, ncol, lane);
    for (int b0 = lane + 64 * 8; b0 < ncol; b0 += 64 * 8) {
      load_tile(m, M, ncol, r, row1, b0);
      fma_tile_k<K>(s, m, vec, ld, ncol, b0);
    }
    if (r + 4 * nw < row1) load_tile(m, M, ncol, r + 4 * nw, row1, lane);
    double v[N];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) v[u * K + k] = s[u][k];
    butterfly_sum<N>(v, lane);
    if (emitter && r + ul < row1) emit(r + ul, kl, v[0]);
  }
}

// k_coarse_fwd for K columns (column k of g_nd, contrib, ybuf and x at
// offsets k * np, k * maxp * np, k * np and k * nc).
template <int K>
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_fwd_k(const CChunk* __restrict__ chunks, const double* __restrict__ fwd,
                   const double* __restrict__ g_nd, double* __restrict__ contrib, int maxp,
                   int np, const int* __restrict__ cdest, double* __restrict__ ybuf,
                   const int* __restrict__ idx, double* __restrict__ x, int nc) {
  extern __shared__ double v[];
  const CChunk ch = chunks[blockIdx.x];
  const int nf = ch.nf;
  const double* M = fwd + ch.mat;
  const int yoff = ch.yoff, coff = ch.coff;
  const long long cstride = (long long)maxp * np;
  int dst = -1;
  auto pre = [&](int row, int) {
    dst = (row >= nf && row < ch.row1) ? cdest[coff + row - nf] : -1;
  };
  double m[4][8];
  const int rw = ch.row0 + 4 * (threadIdx.x >> 6);
  load_tile(m, M, nf, rw, ch.row1, threadIdx.x & 63);
  {
    const int bi = butterfly_index<4 * K>(threadIdx.x & 63);
    pre(rw + bi / K, bi % K);
  }
  for (int e = threadIdx.x; e < nf * K; e += blockDim.x) {
    const int k = e / nf, a = e - k * nf;
    const long long t = (long long)yoff + a;
    double s = g_nd[(long long)k * np + t];
    const double* ck = contrib + k * cstride;
    for (int u0 = 0; u0 < maxp; u0 += 8) {
      double c[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) c[q] = u0 + q < maxp ? ck[(long long)(u0 + q) * np + t] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (u0 + q < maxp) s -= c[q];
    }
    v[k * nf + a] = s;
  }
  __syncthreads();
  gemv_chunk_k<K>(M, nf, ch.row0, ch.row1, v, nf, m, pre, [&](int row, int k, double val) {
    if (row >= nf)
      contrib[k * cstride + dst] = val;
    else if (ch.nu == 0)
      x[(long long)k * nc + idx[ch.fcol + row]] = val;
    else
      ybuf[(long long)k * np + yoff + row] = val;
  });
}

// k_coarse_bwd for K columns (column k of ybuf and x at offsets k * np and
// k * nc).
template <int K>
__global__ void __launch_bounds__(kVecThreads)
    k_coarse_bwd_k(const CChunk* __restrict__ chunks, const double* __restrict__ bwd,
                   const int* __restrict__ idx, const double* __restrict__ ybuf,
                   double* __restrict__ x, int np, int nc) {
  extern __shared__ double xu[];
  const CChunk ch = chunks[blockIdx.x];
  const int nu = ch.nu;
  const double* M = bwd + ch.mat;
  const int yoff = ch.yoff, fcol = ch.fcol;
  int dst = 0;
  double y = 0.0;
  auto pre = [&](int row, int k) {
    if (row < ch.row1) {
      dst = idx[fcol + row];
      y = ybuf[(long long)k * np + yoff + row];
    }
  };
  double m[4][8];
  const int rw = ch.row0 + 4 * (threadIdx.x >> 6);
  load_tile(m, M, nu, rw, ch.row1, threadIdx.x & 63);
  {
    const int bi = butterfly_index<4 * K>(threadIdx.x & 63);
    pre(rw + bi / K, bi % K);
  }
  for (int e = threadIdx.x; e < nu * K; e += blockDim.x) {
    const int k = e / nu, b = e - k * nu;
    xu[k * nu + b] = x[(long long)k * nc + idx[ch.ucol + b]];
  }
  __syncthreads();
  gemv_chunk_k<K>(M, nu, ch.row0, ch.row1, xu, nu, m, pre,
                  [&](int, int k, double val) { x[(long long)k * nc + dst] = y - val; });
}

// k_reconstruct for K columns: p_k[Omega_i] += P_i x_i^k, each MBF entry
// loaded once for all k.
template <typename T, typename S, int K>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct_k(const BoxDesc* __restrict__ boxes, const S* __restrict__ mbf,
                    const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                    const double* __restrict__ xc, int nc, RhsPtrs<T> p, int nx) {
  __shared__ T xs[K][64];
  const int i = blockIdx.x;
  const BoxDesc d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0, ncell = d.obx * d.oby;
  for (int e = threadIdx.x; e < nk * K; e += blockDim.x) {
    const int k = e / nk, j = e - k * nk;
    xs[k][j] = (T)xc[(long long)k * nc + k0 + j];
  }
  __syncthreads();
  const S* P = mbf + mbf_off[i];
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int a = q % d.obx, j = q / d.obx;
    const long long c = (long long)(d.y0 + d.oy + j) * nx + d.x0 + d.ox + a;
    T s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = p.v[k][c];
    for (int j2 = 0; j2 < nk; ++j2) {
      const T pv = (T)P[(long long)j2 * ncell + q];
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] = fmat(pv, xs[k][j2], s[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) p.v[k][c] = s[k];
  }
}

// k_reconstruct_k for 8 right-hand sides on the matrix cores: per
// subdomain, P_i^T (cells x nk, nk <= 8 basis functions) times X (nk x 8
// columns) is added to the 8 columns of p[Omega_i] in tiles of 16 cells, one
// wave per tile, as a 16 x 16 x 8 product (columns 8..15 and basis functions
// past nk are zero).  MfmaRecon selects the instruction: 0 the FP32 or FP64
// 16x16x4 MFMA of the arithmetic type (two steps of four basis functions);
// 1 the BF16 16x16x16 MFMA with FP32 accumulation (P and X rounded to BF16,
// nearest even; FP32 arithmetic only).  The sums are those of the MFMA, not
// of k_reconstruct_k's FMA chain, so results differ from it in rounding.
// MFMA 16 x 16 operand layout: lane l holds A[l % 16][l / 16] (cells x
// basis functions), B[l / 16][l % 16] (basis functions x columns), and in
// accumulator register r row 4 (l / 16) + r of column l % 16 (FP32 and
// BF16 forms) or row 4 r + l / 16 (FP64 form); the BF16 form holds four
// consecutive k per lane (k = 4 (l / 16) .. + 3).
typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));
typedef short mfma_s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
template <typename T, int MODE> struct MfmaAcc;
template <> struct MfmaAcc<float, 0> { typedef mfma_f32x4 type; };
template <> struct MfmaAcc<float, 1> { typedef mfma_f32x4 type; };
template <> struct MfmaAcc<double, 0> { typedef mfma_f64x4 type; };

template <typename T, typename S, int MODE>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct_mfma(const BoxDesc* __restrict__ boxes, const S* __restrict__ mbf,
                       const long long* __restrict__ mbf_off, const int* __restrict__ dof_off,
                       const double* __restrict__ xc, int nc, RhsPtrs<T> p, int nx) {
  typedef typename MfmaAcc<T, MODE>::type Acc;
  __shared__ T xs[16][16];
  const int i = blockIdx.x;
  const BoxDesc d = boxes[i];
  const int k0 = dof_off[i], nk = dof_off[i + 1] - k0, ncell = d.obx * d.oby;
  for (int e = threadIdx.x; e < 16 * 16; e += blockDim.x) {
    const int k = e / 16, j = e % 16;
    xs[k][j] = (k < nk && k < 8 && j < 8) ? (T)xc[(long long)j * nc + k0 + k] : T(0);
  }
  __syncthreads();
  const S* P = mbf + mbf_off[i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  T* pj = p.v[li < 8 ? li : 0];
  const long long base = (long long)(d.y0 + d.oy) * nx + d.x0 + d.ox;
  for (int t = wid; t * 16 < ncell; t += nw) {
    const int q = 16 * t + li;
    long long addr[4];
    bool ok[4];
    Acc c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int qq = 16 * t + (sizeof(T) == 8 ? 4 * r + lk : 4 * lk + r);
      ok[r] = li < 8 && qq < ncell;
      const int qc = qq < ncell ? qq : 0;
      const int row = qc / d.obx, col = qc - row * d.obx;
      addr[r] = base + (long long)row * nx + col;
      c[r] = ok[r] ? pj[addr[r]] : T(0);
    }
    if constexpr (MODE == 0) {
#pragma unroll
      for (int s4 = 0; s4 < 2; ++s4) {
        const int k = 4 * s4 + lk;
        const T a = (k < nk && q < ncell) ? (T)P[(long long)k * ncell + q] : T(0);
        const T b = xs[k][li];
        if constexpr (sizeof(T) == 4)
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        else
          c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
      }
    } else {
      mfma_s16x4 a, b;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * lk + u;
        a[u] = bf16_rne((k < nk && q < ncell) ? (float)P[(long long)k * ncell + q] : 0.0f);
        b[u] = bf16_rne((float)xs[k][li]);
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (ok[r]) pj[addr[r]] = c[r];
  }
}

// Smoothing residuals rho_k = r_k - A p_k (blockIdx.y = k).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_residual_k(const T* __restrict__ tx, const T* __restrict__ ty, int nx, int ny,
                 RhsPtrs<const double> r, RhsPtrs<const T> p, RhsPtrs<T> rho) {
  const long long n = (long long)nx * ny;
  const double* rk = r.v[blockIdx.y];
  const T* pk = p.v[blockIdx.y];
  T* ok = rho.v[blockIdx.y];
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int iy = (int)(c / nx), ix = (int)(c - (long long)iy * nx);
    ok[c] = (T)rk[c] - stencil(tx, ty, nx, ny, ix, iy, pk);
  }
}

// k_sum for K vectors (blockIdx.y = k; partials of k at k * kMaxVecBlocks).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_sum_k(RhsPtrs<const T> p, long long n, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  const T* pk = p.v[blockIdx.y];
  const long long st = (long long)gridDim.x * blockDim.x;
  double s = 0.0;
  for (long long c0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; c0 < n;
       c0 += kRound * st) {
    T a[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = pk[c < n ? c : n - 1];
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
      if (c0 + u * st < n) s += (double)a[u];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * kMaxVecBlocks + blockIdx.x] = s;
}

// k_finalize for K vectors (blockIdx.y = k).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_finalize_k(RhsPtrs<const T> p, long long n, const double* __restrict__ partials, int nb,
                 RhsPtrs<double> z) {
  __shared__ double red[kVecThreads / 64];
  const T* pk = p.v[blockIdx.y];
  double* zk = z.v[blockIdx.y];
  const double* part = partials ? partials + (long long)blockIdx.y * kMaxVecBlocks : nullptr;
  const long long st = (long long)gridDim.x * blockDim.x;
  T a[kRound];
  auto load = [&](long long c0) {
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      a[u] = pk[c < n ? c : n - 1];
    }
  };
  const long long start = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  load(start);
  const double mean = part ? reduce_partials(part, nb, red) / (double)n : 0.0;
  for (long long c0 = start; c0 < n; c0 += kRound * st) {
    if (c0 != start) load(c0);
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const long long c = c0 + u * st;
      if (c < n) zk[c] = (double)a[u] - mean;
    }
  }
}

inline int grid_for(long long n) {
  long long b = (n + kVecThreads - 1) / kVecThreads;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void launch_op_apply(const double* tx, const double* ty, int nx, int ny, const double* x,
                     double* y, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_op_apply, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny, x,
                     y);
}

void launch_rhs(const double* tx, const double* ty, int nx, int ny, const int* bc,
                const double* f, const double* g, double h, double* b, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny, bc[0],
                     bc[1], bc[2], bc[3], f, g, h, b);
}

// Column-buffer width (registers) and lane-group size for boxes up to max_bx
// cells wide.
inline int col_width(int max_bx) { return box_cols(max_bx); }
inline int group_size(int max_bx) { return max_bx <= 16 ? 16 : max_bx <= 32 ? 32 : 64; }
// Words of a group's vector slot (vec_words of the kernels).
inline int vec_slot_words(int max_bx) {
  return (col_width(max_bx) / 2 + 2 * group_size(max_bx) + 3) / 4 * 4;
}
// Words of S in 16 bytes; x rounded up to a multiple of them.
inline int round16(long long x, size_t w) {
  const long long e = 16 / (long long)w;
  return (int)((x + e - 1) / e * e);
}
// LDS bytes of one lane group: broadcast slot and box (arithmetic words t)
// and the couplings (storage words w), rounded to 16 bytes.
inline size_t group_bytes(int max_bx, int max_cells, size_t t, size_t w) {
  const size_t b = (size_t)vec_slot_words(max_bx) * t + (size_t)round16(max_cells, w) * w +
                   (size_t)max_cells * t;
  return (b + 15) / 16 * 16;
}
// Lane groups per workgroup: up to 256 threads, fewer when the boxes' LDS
// would exceed 64 KB (0 when even one group does not fit).
int box_groups(int max_bx, int max_cells, size_t t, size_t w) {
  const int gs = group_size(max_bx);
  for (int groups = kBoxThreads / gs; groups >= 1; groups /= 2)
    if (groups * group_bytes(max_bx, max_cells, t, w) <= 64 * 1024) return groups;
  return 0;
}
size_t box_lds_bytes(int max_bx, int max_cells, size_t t, size_t w) {
  const int groups = box_groups(max_bx, max_cells, t, w);
  return groups ? groups * group_bytes(max_bx, max_cells, t, w) : ~(size_t)0;
}
#define MRCM_BOX_DISPATCH(KERNEL, T, S, max_bx, ...)                                      \
  do {                                                                                   \
    switch (col_width(max_bx)) {                                                         \
      case 16: hipLaunchKernelGGL((KERNEL<T, S, 16>), __VA_ARGS__); break;               \
      case 20: hipLaunchKernelGGL((KERNEL<T, S, 20>), __VA_ARGS__); break;               \
      case 24: hipLaunchKernelGGL((KERNEL<T, S, 24>), __VA_ARGS__); break;               \
      case 32: hipLaunchKernelGGL((KERNEL<T, S, 32>), __VA_ARGS__); break;               \
      case 36: hipLaunchKernelGGL((KERNEL<T, S, 36>), __VA_ARGS__); break;               \
      case 40: hipLaunchKernelGGL((KERNEL<T, S, 40>), __VA_ARGS__); break;               \
      case 48: hipLaunchKernelGGL((KERNEL<T, S, 48>), __VA_ARGS__); break;               \
      default: hipLaunchKernelGGL((KERNEL<T, S, 64>), __VA_ARGS__); break;               \
    }                                                                                    \
  } while (0)
template <typename T, typename S>
void launch_local(const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                  const S* coup, const double* r, T* p, int nx, const int* dof_off,
                  const int* dof_side, const int* dof_q, const int* dof_face0,
                  const double* face_w, double* mU, double* mP, hipStream_t s, int groups_cap) {
  int groups = box_groups(max_bx, max_cells, sizeof(T), sizeof(S));
  if (groups_cap > 0 && groups_cap < groups) groups = groups_cap;
  const int gb = (int)group_bytes(max_bx, max_cells, sizeof(T), sizeof(S));
  const size_t shm = (size_t)groups * gb;
  const int cp_words = round16(max_cells, sizeof(S));
  const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
  MRCM_BOX_DISPATCH(k_local, T, S, max_bx, grid, block, shm, s, boxes, m, gb, cp_words,
                    dinv, coup, r, p, nx, dof_off, dof_side, dof_q, dof_face0, face_w, mU, mP);
}

void launch_coarse_rhs(const int4* gsrc, const double* gscale, const double* mU,
                       const double* mP, double* g_nd, int np, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_coarse_rhs, dim3((np + 255) / 256), dim3(256), 0, s, gsrc, gscale, mU, mP,
                     g_nd, np);
}
void launch_coarse_resid(int k, const int* rp, const int* ci, const double* v,
                         const double* g_nd, const double* x, double* r_nd, int np, int nc,
                         hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_coarse_resid, dim3((np + 255) / 256, k), dim3(256), 0, s, rp, ci, v, g_nd,
                     x, r_nd, np, nc);
}
void launch_coarse_add(double* x, const double* dx, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_coarse_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, dx, n);
}

// Threads per chunk of an interface level: levels with very many chunks
// (the leaves: small fronts) take one wave per chunk, which takes its chunk
// whole, so that every chunk of the level is resident at once; the other
// levels take four waves per chunk (a sweep of the threshold over 0, 1024,
// 2048 and never found 2048 best at 1024^2 and 4096^2).
int coarse_threads(int nchunks, bool forward) {
  return forward || nchunks < 2048 ? kVecThreads : 64;
}

void launch_coarse_fwd(const CChunk* chunks, int nchunks, const double* fwd, const double* g_nd,
                       double* contrib, int maxp, int np, const int* cdest, double* ybuf,
                       const int* idx, double* x, int max_nf, hipStream_t s, int threads) {
  if (nchunks <= 0) return;
  if (threads != 64 && threads != kVecThreads) threads = coarse_threads(nchunks, true);
  hipLaunchKernelGGL(k_coarse_fwd, dim3(nchunks), dim3(threads),
                     sizeof(double) * (size_t)(max_nf > 0 ? max_nf : 1), s, chunks, fwd, g_nd,
                     contrib, maxp, np, cdest, ybuf, idx, x);
}
void launch_coarse_bwd(const CChunk* chunks, int nchunks, const double* bwd, const int* idx,
                       const double* ybuf, double* x, int max_nu, hipStream_t s, int threads) {
  if (nchunks <= 0) return;
  if (threads != 64 && threads != kVecThreads) threads = coarse_threads(nchunks, false);
  hipLaunchKernelGGL(k_coarse_bwd, dim3(nchunks), dim3(threads),
                     sizeof(double) * (size_t)(max_nu > 0 ? max_nu : 1), s, chunks, bwd, idx,
                     ybuf, x);
}
template <typename T, typename S>
void launch_reconstruct(const BoxDesc* boxes, int m, const S* mbf, const long long* mbf_off,
                        const int* dof_off, const double* xc, T* p, int nx, hipStream_t s) {
  hipLaunchKernelGGL((k_reconstruct<T, S>), dim3(m), dim3(kBoxThreads), 0, s, boxes, mbf,
                     mbf_off, dof_off, xc, p, nx);
}

template <typename T>
void launch_residual(const T* tx, const T* ty, int nx, int ny, const double* r, const T* p,
                     T* rho, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_residual<T>, dim3(grid_for(n)), dim3(kVecThreads), 0, s, tx, ty, nx, ny,
                     r, p, rho);
}

template <typename T, typename S>
void launch_patch(const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                  const S* coup, const T* rho, T* p, int nx, hipStream_t s, int groups_cap) {
  int groups = box_groups(max_bx, max_cells, sizeof(T), sizeof(S));
  if (groups_cap > 0 && groups_cap < groups) groups = groups_cap;
  const int gb = (int)group_bytes(max_bx, max_cells, sizeof(T), sizeof(S));
  const size_t shm = (size_t)groups * gb;
  const int cp_words = round16(max_cells, sizeof(S));
  const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
  MRCM_BOX_DISPATCH(k_patch, T, S, max_bx, grid, block, shm, s, boxes, m, gb, cp_words,
                    dinv, coup, rho, p, nx);
}

// ---- K right-hand sides per launch ----
namespace {
template <typename T>
RhsPtrs<T> rhs_ptrs(int k, T* const* v) {
  RhsPtrs<T> out{};
  for (int i = 0; i < k; ++i) out.v[i] = v[i];
  return out;
}
void check_k(int k) {
  if (k != 2 && k != 4 && k != 8)
    throw Error(MRCM_EINVAL, "multi-RHS launch of unsupported width");
}
inline size_t group_bytes_k(int k, int max_bx, int max_cells, size_t t, size_t w) {
  const size_t b = (size_t)k * vec_slot_words(max_bx) * t + (size_t)round16(max_cells, w) * w;
  return (b + 15) / 16 * 16;
}
int box_groups_k(int k, int max_bx, int max_cells, size_t t, size_t w) {
  const int gs = group_size(max_bx);
  for (int groups = kBoxThreads / gs; groups >= 1; groups /= 2)
    if (groups * group_bytes_k(k, max_bx, max_cells, t, w) <= 64 * 1024) return groups;
  return 0;
}
}  // namespace

size_t box_lds_bytes_k(int k, int max_bx, int max_cells, size_t t, size_t w) {
  const int groups = box_groups_k(k, max_bx, max_cells, t, w);
  return groups ? groups * group_bytes_k(k, max_bx, max_cells, t, w) : ~(size_t)0;
}

// Right-hand sides one box launch takes at most, by column width: what the
// lane's registers hold without spilling (quads in flight, four partial sums
// and the rows of every column); 1 = the one-RHS kernels, once per column.
inline int box_width_k(int nb, size_t w) {
  if (w == 8) return nb <= 16 ? 4 : nb <= 48 ? 2 : 1;
  return nb <= 16 ? 8 : nb <= 32 ? 4 : nb <= 48 ? 2 : 1;
}

#define MRCM_BOX_DISPATCH_K(KERNEL, T, S, nb, kk, ...)                                  \
  do {                                                                                 \
    if (nb == 16 && kk == 8) hipLaunchKernelGGL((KERNEL<T, S, 16, 8>), __VA_ARGS__);   \
    else if (nb == 16 && kk == 4) hipLaunchKernelGGL((KERNEL<T, S, 16, 4>), __VA_ARGS__); \
    else if (nb == 16) hipLaunchKernelGGL((KERNEL<T, S, 16, 2>), __VA_ARGS__);         \
    else if (nb == 20 && kk == 4) hipLaunchKernelGGL((KERNEL<T, S, 20, 4>), __VA_ARGS__); \
    else if (nb == 20) hipLaunchKernelGGL((KERNEL<T, S, 20, 2>), __VA_ARGS__);         \
    else if (nb == 24 && kk == 4) hipLaunchKernelGGL((KERNEL<T, S, 24, 4>), __VA_ARGS__); \
    else if (nb == 24) hipLaunchKernelGGL((KERNEL<T, S, 24, 2>), __VA_ARGS__);         \
    else if (nb == 32 && kk == 4) hipLaunchKernelGGL((KERNEL<T, S, 32, 4>), __VA_ARGS__); \
    else if (nb == 32) hipLaunchKernelGGL((KERNEL<T, S, 32, 2>), __VA_ARGS__);         \
    else if (nb == 36) hipLaunchKernelGGL((KERNEL<T, S, 36, 2>), __VA_ARGS__);         \
    else if (nb == 40) hipLaunchKernelGGL((KERNEL<T, S, 40, 2>), __VA_ARGS__);         \
    else hipLaunchKernelGGL((KERNEL<T, S, 48, 2>), __VA_ARGS__);                       \
  } while (0)
#define MRCM_K_DISPATCH(k, CALL) \
  do {                           \
    if ((k) == 2) {              \
      constexpr int K = 2;       \
      CALL;                      \
    } else if ((k) == 4) {       \
      constexpr int K = 4;       \
      CALL;                      \
    } else {                     \
      constexpr int K = 8;       \
      CALL;                      \
    }                            \
  } while (0)

template <typename T, typename S>
void launch_local_k(int k, const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                    const S* coup, const double* const* r, T* const* p, T* const* e, int nx,
                    const int* dof_off, const int* dof_side, const int* dof_q,
                    const int* dof_face0, const double* face_w, double* mU, double* mP, int nc,
                    hipStream_t s) {
  check_k(k);
  const int nb = col_width(max_bx), kk = std::min(k, box_width_k(nb, sizeof(S)));
  for (int k0 = 0; k0 < k; k0 += kk) {
    double* u = mU + (long long)k0 * nc;
    double* v = mP + (long long)k0 * nc;
    if (kk == 1) {
      launch_local<T, S>(boxes, m, max_cells, max_bx, dinv, coup, r[k0], p[k0], nx, dof_off,
                         dof_side, dof_q, dof_face0, face_w, u, v, s);
      continue;
    }
    const int groups = box_groups_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const size_t shm = box_lds_bytes_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const int gb = (int)group_bytes_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
    const RhsPtrs<const double> rp = rhs_ptrs(kk, r + k0);
    const RhsPtrs<T> pp = rhs_ptrs(kk, p + k0), ep = rhs_ptrs(kk, e + k0);
    MRCM_BOX_DISPATCH_K(k_local_k, T, S, nb, kk, grid, block, shm, s, boxes, m, gb, dinv, coup,
                        rp, pp, ep, nx, dof_off, dof_side, dof_q, dof_face0, face_w, u, v, nc);
  }
}

void launch_coarse_rhs_k(int k, const int4* gsrc, const double* gscale, const double* mU,
                         const double* mP, double* g_nd, int np, int nc, hipStream_t s) {
  check_k(k);
  if (np <= 0) return;
  hipLaunchKernelGGL(k_coarse_rhs_k, dim3((np + 255) / 256, k), dim3(256), 0, s, gsrc, gscale,
                     mU, mP, g_nd, np, nc);
}

// Columns go in groups of at most 4 (wider ones spill registers) whose LDS
// vector (group width x the largest front) fits in 64 KB.
static int coarse_width(int k, int max_dim) {
  int w = k < 4 ? k : 4;
  while (w > 1 && (size_t)w * (max_dim > 0 ? max_dim : 1) * sizeof(double) > 64 * 1024) w /= 2;
  return w;
}

void launch_coarse_fwd_k(int k, const CChunk* chunks, int nchunks, const double* fwd,
                         const double* g_nd, double* contrib, int maxp, int np, const int* cdest,
                         double* ybuf, const int* idx, double* x, int nc, int max_nf,
                         hipStream_t s) {
  check_k(k);
  if (nchunks <= 0) return;
  const int w = coarse_width(k, max_nf);
  for (int k0 = 0; k0 < k; k0 += w) {
    const double* g = g_nd + (long long)k0 * np;
    double* c = contrib + (long long)k0 * maxp * np;
    double* y = ybuf + (long long)k0 * np;
    double* xk = x + (long long)k0 * nc;
    const size_t shm = sizeof(double) * (size_t)w * (max_nf > 0 ? max_nf : 1);
    const dim3 grid(nchunks), block(coarse_threads(nchunks, true));
    if (w == 1)
      hipLaunchKernelGGL(k_coarse_fwd, grid, block, shm, s, chunks, fwd, g, c, maxp, np, cdest, y,
                         idx, xk);
    else if (w == 2)
      hipLaunchKernelGGL(k_coarse_fwd_k<2>, grid, block, shm, s, chunks, fwd, g, c, maxp, np, cdest,
                         y, idx, xk, nc);
    else
      hipLaunchKernelGGL(k_coarse_fwd_k<4>, grid, block, shm, s, chunks, fwd, g, c, maxp, np, cdest,
                         y, idx, xk, nc);
  }
}

void launch_coarse_bwd_k(int k, const CChunk* chunks, int nchunks, const double* bwd,
                         const int* idx, const double* ybuf, double* x, int max_nu, int np, int nc,
                         hipStream_t s) {
  check_k(k);
  if (nchunks <= 0) return;
  const int w = coarse_width(k, max_nu);
  for (int k0 = 0; k0 < k; k0 += w) {
    const double* y = ybuf + (long long)k0 * np;
    double* xk = x + (long long)k0 * nc;
    const size_t shm = sizeof(double) * (size_t)w * (max_nu > 0 ? max_nu : 1);
    const dim3 grid(nchunks), block(coarse_threads(nchunks, false));
    if (w == 1)
      hipLaunchKernelGGL(k_coarse_bwd, grid, block, shm, s, chunks, bwd, idx, y, xk);
    else if (w == 2)
      hipLaunchKernelGGL(k_coarse_bwd_k<2>, grid, block, shm, s, chunks, bwd, idx, y, xk, np, nc);
    else
      hipLaunchKernelGGL(k_coarse_bwd_k<4>, grid, block, shm, s, chunks, bwd, idx, y, xk, np, nc);
  }
}

template <typename T, typename S>
void launch_reconstruct_k(int k, const BoxDesc* boxes, int m, const S* mbf,
                          const long long* mbf_off, const int* dof_off, const double* xc, int nc,
                          T* const* p, int nx, hipStream_t s) {
  check_k(k);
  const RhsPtrs<T> pp = rhs_ptrs(k, p);
  MRCM_K_DISPATCH(k, hipLaunchKernelGGL((k_reconstruct_k<T, S, K>), dim3(m), dim3(kBoxThreads), 0,
                                        s, boxes, mbf, mbf_off, dof_off, xc, nc, pp, nx));
}

template <typename T, typename S>
void launch_reconstruct_mfma(int mode, const BoxDesc* boxes, int m, const S* mbf,
                             const long long* mbf_off, const int* dof_off, const double* xc,
                             int nc, T* const* p, int nx, hipStream_t s) {
  const RhsPtrs<T> pp = rhs_ptrs(8, p);
  if constexpr (sizeof(T) == 4) {
    if (mode == 2) {
      hipLaunchKernelGGL((k_reconstruct_mfma<T, S, 1>), dim3(m), dim3(kBoxThreads), 0, s, boxes,
                         mbf, mbf_off, dof_off, xc, nc, pp, nx);
      return;
    }
  }
  hipLaunchKernelGGL((k_reconstruct_mfma<T, S, 0>), dim3(m), dim3(kBoxThreads), 0, s, boxes, mbf,
                     mbf_off, dof_off, xc, nc, pp, nx);
}

template <typename T>
void launch_residual_k(int k, const T* tx, const T* ty, int nx, int ny, const double* const* r,
                       const T* const* p, T* const* rho, hipStream_t s) {
  check_k(k);
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_residual_k<T>, dim3(grid_for(n), k), dim3(kVecThreads), 0, s, tx, ty, nx,
                     ny, rhs_ptrs(k, r), rhs_ptrs(k, p), rhs_ptrs(k, rho));
}

template <typename T, typename S>
void launch_patch_k(int k, const BoxDesc* boxes, int m, int max_cells, int max_bx, const S* dinv,
                    const S* coup, const T* const* rho, T* const* p, T* const* e, int nx,
                    hipStream_t s) {
  check_k(k);
  const int nb = col_width(max_bx), kk = std::min(k, box_width_k(nb, sizeof(S)));
  for (int k0 = 0; k0 < k; k0 += kk) {
    if (kk == 1) {
      launch_patch<T, S>(boxes, m, max_cells, max_bx, dinv, coup, rho[k0], p[k0], nx, s);
      continue;
    }
    const int groups = box_groups_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const size_t shm = box_lds_bytes_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const int gb = (int)group_bytes_k(kk, max_bx, max_cells, sizeof(T), sizeof(S));
    const dim3 grid((m + groups - 1) / groups), block(groups * group_size(max_bx));
    const RhsPtrs<const T> rp = rhs_ptrs(kk, rho + k0);
    const RhsPtrs<T> pp = rhs_ptrs(kk, p + k0), ep = rhs_ptrs(kk, e + k0);
    MRCM_BOX_DISPATCH_K(k_patch_k, T, S, nb, kk, grid, block, shm, s, boxes, m, gb, dinv, coup,
                        rp, pp, ep, nx);
  }
}

template <typename T>
void launch_finalize_k(int k, const T* const* p, long long n, int noflow, double* const* z,
                       double* partials, hipStream_t s) {
  check_k(k);
  const int nb = vec_blocks(n);
  const RhsPtrs<const T> pp = rhs_ptrs(k, p);
  if (noflow)
    hipLaunchKernelGGL(k_sum_k<T>, dim3(nb, k), dim3(kVecThreads), 0, s, pp, n, partials);
  hipLaunchKernelGGL(k_finalize_k<T>, dim3(nb, k), dim3(kVecThreads), 0, s, pp, n,
                     noflow ? partials : (const double*)nullptr, nb, rhs_ptrs(k, z));
}

template <typename T>
void launch_finalize(const T* p, long long n, int noflow, double* z, double* partials,
                     hipStream_t s) {
  const int nb = vec_blocks(n);
  if (noflow) hipLaunchKernelGGL(k_sum<T>, dim3(nb), dim3(kVecThreads), 0, s, p, n, partials);
  hipLaunchKernelGGL(k_finalize<T>, dim3(nb), dim3(kVecThreads), 0, s, p, n,
                     noflow ? partials : (const double*)nullptr, nb, z);
}

void launch_convert(const double* src, float* dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(n)), dim3(kVecThreads), 0, s, src, dst, n);
}

void launch_resid_norm(const double* tx, const double* ty, int nx, int ny, const double* b,
                       const double* p, double* r, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_norm, dim3(nb), dim3(kVecThreads), 0, s, tx, ty, nx, ny, b, p, r,
                     partials);
}

void launch_zero(double* v, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kVecThreads), 0, s, v, n);
}

void launch_scale(double* v, long long n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kVecThreads), 0, s, v, n, alpha);
}

void launch_arnoldi_start(const double* tx, const double* ty, int nx, int ny, const double* z,
                          double* w, const double* v0, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_start, dim3(nb), dim3(kVecThreads), 0, s, tx, ty, nx, ny, z, w, v0,
                     partials);
}

void launch_mgs_step(const double* part_in, double* part_out, int nb, double* hcol, int i,
                     double* w, const double* vi, const double* vnext, long long n,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_step, dim3(nb), dim3(kVecThreads), 0, s, part_in, part_out, nb, hcol, i,
                     w, vi, vnext, n);
}

void launch_norm_scale(const double* part_in, int nb, double* hcol, int j, double* w,
                       long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_scale, dim3(nb), dim3(kVecThreads), 0, s, part_in, nb, hcol, j, w, n);
}

void launch_update(double* p, const double* Z, const double* y, int k, long long n,
                   hipStream_t s) {
  // in slices of kMaxUpdate vectors: p is updated in the same order
  for (int i0 = 0; i0 < k; i0 += kMaxUpdate)
    hipLaunchKernelGGL(k_update, dim3(grid_for(n)), dim3(kVecThreads), 0, s, p,
                       Z + (long long)i0 * n, y + i0, k - i0 < kMaxUpdate ? k - i0 : kMaxUpdate, n);
}

void launch_sumsq(const double* x, long long n, double* partials, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(kVecThreads), 0, s, x, n, partials);
}

// ---- launches over several contexts ----------------------------------------
namespace {

// The column whose workgroup range [pre[c], pre[c + 1]) holds workgroup b
// (the largest c with pre[c] <= b; empty ranges are skipped).
__device__ __forceinline__ int many_col(const int* __restrict__ pre, int ncol, int b) {
  int lo = 0, hi = ncol - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ Blk many_blk(const int* __restrict__ pre, int c) {
  return Blk{(int)blockIdx.x - pre[c], pre[c + 1] - pre[c]};
}

template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_local_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol,
                 int group_bytes, int cp_words) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  local_body<T, S, NB, GS>(many_blk(pre, c), a.lbox, a.m, group_bytes, cp_words,
                           static_cast<const S*>(a.ldinv), static_cast<const S*>(a.lcoup), a.r,
                           static_cast<T*>(a.p), a.nx, a.dof_off, a.dof_side, a.dof_q,
                           a.dof_face0, a.face_w, a.mU, a.mP);
}

__global__ void k_coarse_rhs_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre,
                                  int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  coarse_rhs_body(many_blk(pre, c), a.gsrc, a.gscale, a.mU, a.mP, a.g_nd, a.np);
}

__global__ void __launch_bounds__(kVecThreads)
    k_coarse_fwd_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre,
                      const int* __restrict__ first, int ncol, int refine) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  const int q = first[c] + (int)blockIdx.x - pre[c];
  coarse_fwd_body(a.chunks[q], a.cfwd, refine ? a.rnd : a.g_nd, a.contrib, a.maxp, a.np,
                  a.cdest, a.ybuf, a.cidx, refine ? a.dx : a.xc);
}

__global__ void __launch_bounds__(kVecThreads)
    k_coarse_bwd_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre,
                      const int* __restrict__ first, int ncol, int refine) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  const int q = first[c] + (int)blockIdx.x - pre[c];
  coarse_bwd_body(a.chunks[q], a.cbwd, a.cidx, a.ybuf, refine ? a.dx : a.xc);
}

__global__ void k_coarse_resid_many(const ManyCol* __restrict__ cols,
                                    const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  coarse_resid_body(many_blk(pre, c), 0, a.crp, a.cci, a.cv, a.g_nd, a.xc, a.rnd, a.np, a.nc);
}

__global__ void k_coarse_add_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre,
                                  int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  coarse_add_body(many_blk(pre, c), a.xc, a.dx, a.nc);
}

template <typename T, typename S>
__global__ void __launch_bounds__(kBoxThreads)
    k_reconstruct_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  reconstruct_body<T, S>(many_blk(pre, c), a.lbox, static_cast<const S*>(a.mbf), a.mbf_off,
                         a.dof_off, a.xc, static_cast<T*>(a.p), a.nx);
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_residual_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  residual_body<T>(many_blk(pre, c), static_cast<const T*>(a.txT), static_cast<const T*>(a.tyT),
                   a.nx, a.ny, a.r, static_cast<const T*>(a.p), static_cast<T*>(a.rho));
}

template <typename T, typename S, int NB, int GS = (NB <= 16 ? 16 : NB <= 32 ? 32 : 64)>
__global__ void __launch_bounds__(kBoxThreads)
    k_patch_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol,
                 int group_bytes, int cp_words) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  patch_body<T, S, NB, GS>(many_blk(pre, c), a.pbox, a.m, group_bytes, cp_words,
                           static_cast<const S*>(a.pdinv), static_cast<const S*>(a.pcoup),
                           static_cast<const T*>(a.rho), static_cast<T*>(a.p), a.nx);
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_sum_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  sum_body<T>(many_blk(pre, c), static_cast<const T*>(a.p), a.n, a.partials);
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_finalize_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  finalize_body<T>(many_blk(pre, c), static_cast<const T*>(a.p), a.n,
                   a.noflow ? a.partials : (const double*)nullptr, a.nb, a.z);
}

__global__ void __launch_bounds__(kVecThreads)
    k_arnoldi_start_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre,
                         int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  arnoldi_start_body(many_blk(pre, c), a.tx, a.ty, a.nx, a.ny, a.Z + (long long)a.j * a.n,
                     a.V + (long long)(a.j + 1) * a.n, a.V, a.parts);
}

__global__ void __launch_bounds__(kVecThreads)
    k_mgs_step_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol,
                    int i) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  const long long n = a.n;
  mgs_step_body(many_blk(pre, c), a.parts + (i % 2) * kMaxVecBlocks,
                a.parts + ((i + 1) % 2) * kMaxVecBlocks, a.nb, a.hcol, i,
                a.V + (long long)(a.j + 1) * n, a.V + (long long)i * n,
                i < a.j ? a.V + (long long)(i + 1) * n : (const double*)nullptr, n);
}

__global__ void __launch_bounds__(kVecThreads)
    k_norm_scale_many(const ManyCol* __restrict__ cols, const int* __restrict__ pre, int ncol) {
  const int c = many_col(pre, ncol, blockIdx.x);
  const ManyCol& a = cols[c];
  norm_scale_body(many_blk(pre, c), a.parts + ((a.j + 1) % 2) * kMaxVecBlocks, a.nb, a.hcol,
                  a.j + 1, a.V + (long long)(a.j + 1) * a.n, a.n);
}

// One workgroup per item.
__global__ void k_gather(const GatherItem* __restrict__ items, double* __restrict__ stage) {
  const GatherItem g = items[blockIdx.x];
  for (int e = threadIdx.x; e < g.count; e += blockDim.x) stage[g.dst + e] = g.src[e];
}

}  // namespace

template <typename T, typename S>
void launch_local_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int max_cells,
                       int max_bx, hipStream_t s) {
  if (blocks <= 0) return;
  const int groups = box_groups(max_bx, max_cells, sizeof(T), sizeof(S));
  const int gb = (int)group_bytes(max_bx, max_cells, sizeof(T), sizeof(S));
  const int cp_words = round16(max_cells, sizeof(S));
  MRCM_BOX_DISPATCH(k_local_many, T, S, max_bx, dim3(blocks), dim3(groups * group_size(max_bx)),
                    (size_t)groups * gb, s, cols, pre, ncol, gb, cp_words);
}
void launch_coarse_rhs_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_coarse_rhs_many, dim3(blocks), dim3(256), 0, s, cols, pre, ncol);
}
void launch_coarse_fwd_many(const ManyCol* cols, const int* pre, const int* first, int ncol,
                            int blocks, int refine, int max_nf, hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_coarse_fwd_many, dim3(blocks), dim3(coarse_threads(blocks, true)),
                     sizeof(double) * (size_t)(max_nf > 0 ? max_nf : 1), s, cols, pre, first,
                     ncol, refine);
}
void launch_coarse_bwd_many(const ManyCol* cols, const int* pre, const int* first, int ncol,
                            int blocks, int refine, int max_nu, hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_coarse_bwd_many, dim3(blocks), dim3(coarse_threads(blocks, false)),
                     sizeof(double) * (size_t)(max_nu > 0 ? max_nu : 1), s, cols, pre, first,
                     ncol, refine);
}
void launch_coarse_resid_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                              hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_coarse_resid_many, dim3(blocks), dim3(256), 0, s, cols, pre, ncol);
}
void launch_coarse_add_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_coarse_add_many, dim3(blocks), dim3(256), 0, s, cols, pre, ncol);
}
template <typename T, typename S>
void launch_reconstruct_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                             hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL((k_reconstruct_many<T, S>), dim3(blocks), dim3(kBoxThreads), 0, s, cols,
                     pre, ncol);
}
template <typename T>
void launch_residual_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                          hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_residual_many<T>, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre, ncol);
}
template <typename T, typename S>
void launch_patch_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int max_cells,
                       int max_bx, hipStream_t s) {
  if (blocks <= 0) return;
  const int groups = box_groups(max_bx, max_cells, sizeof(T), sizeof(S));
  const int gb = (int)group_bytes(max_bx, max_cells, sizeof(T), sizeof(S));
  const int cp_words = round16(max_cells, sizeof(S));
  MRCM_BOX_DISPATCH(k_patch_many, T, S, max_bx, dim3(blocks), dim3(groups * group_size(max_bx)),
                    (size_t)groups * gb, s, cols, pre, ncol, gb, cp_words);
}
template <typename T>
void launch_sum_many(const ManyCol* cols, const int* pre, int ncol, int blocks, hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_sum_many<T>, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre, ncol);
}
template <typename T>
void launch_finalize_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                          hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_finalize_many<T>, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre, ncol);
}
void launch_arnoldi_start_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                               hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_arnoldi_start_many, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre,
                     ncol);
}
void launch_mgs_step_many(const ManyCol* cols, const int* pre, int ncol, int blocks, int i,
                          hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_mgs_step_many, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre, ncol, i);
}
void launch_norm_scale_many(const ManyCol* cols, const int* pre, int ncol, int blocks,
                            hipStream_t s) {
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_norm_scale_many, dim3(blocks), dim3(kVecThreads), 0, s, cols, pre, ncol);
}
void launch_gather(const GatherItem* items, int count, double* stage, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(count), dim3(64), 0, s, items, stage);
}

#define MRCM_INSTANTIATE_TS(T, S)                                                              \
  template void launch_local<T, S>(const BoxDesc*, int, int, int, const S*, const S*,          \
                                   const double*, T*, int, const int*, const int*, const int*,   \
                                   const int*, const double*, double*, double*, hipStream_t,     \
                                   int);                                                        \
  template void launch_reconstruct<T, S>(const BoxDesc*, int, const S*, const long long*,       \
                                         const int*, const double*, T*, int, hipStream_t);      \
  template void launch_patch<T, S>(const BoxDesc*, int, int, int, const S*, const S*,          \
                                   const T*, T*, int, hipStream_t, int);                         \
  template void launch_local_k<T, S>(int, const BoxDesc*, int, int, int, const S*, const S*,    \
                                     const double* const*, T* const*, T* const*, int,           \
                                     const int*, const int*, const int*, const int*,            \
                                     const double*, double*, double*, int, hipStream_t);        \
  template void launch_reconstruct_k<T, S>(int, const BoxDesc*, int, const S*,                  \
                                           const long long*, const int*, const double*, int,    \
                                           T* const*, int, hipStream_t);                        \
  template void launch_reconstruct_mfma<T, S>(int, const BoxDesc*, int, const S*,               \
                                              const long long*, const int*, const double*, int, \
                                              T* const*, int, hipStream_t);                     \
  template void launch_patch_k<T, S>(int, const BoxDesc*, int, int, int, const S*, const S*,    \
                                     const T* const*, T* const*, T* const*, int, hipStream_t); \
  template void launch_local_many<T, S>(const ManyCol*, const int*, int, int, int, int,         \
                                        hipStream_t);                                           \
  template void launch_reconstruct_many<T, S>(const ManyCol*, const int*, int, int, hipStream_t); \
  template void launch_patch_many<T, S>(const ManyCol*, const int*, int, int, int, int,         \
                                        hipStream_t);
#define MRCM_INSTANTIATE_T(T)                                                                  \
  template void launch_residual<T>(const T*, const T*, int, int, const double*, const T*, T*,   \
                                   hipStream_t);                                                \
  template void launch_finalize<T>(const T*, long long, int, double*, double*, hipStream_t);    \
  template void launch_residual_k<T>(int, const T*, const T*, int, int, const double* const*,   \
                                     const T* const*, T* const*, hipStream_t);                  \
  template void launch_finalize_k<T>(int, const T* const*, long long, int, double* const*,      \
                                     double*, hipStream_t);                                     \
  template void launch_residual_many<T>(const ManyCol*, const int*, int, int, hipStream_t);     \
  template void launch_sum_many<T>(const ManyCol*, const int*, int, int, hipStream_t);          \
  template void launch_finalize_many<T>(const ManyCol*, const int*, int, int, hipStream_t);

MRCM_INSTANTIATE_TS(double, double)
MRCM_INSTANTIATE_TS(float, float)
MRCM_INSTANTIATE_TS(double, float)
MRCM_INSTANTIATE_T(double)
MRCM_INSTANTIATE_T(float)

}  // namespace mrcm
