// gfx950 kernels of the tree-cotree gauged IETI-DP hot path.
//
// Factor side: batched right-looking tile Cholesky over 64x64 FP64 tiles
// (column-major inside a tile) of every subdomain's augmented matrix,
// driven by host-built task lists: one launch per kernel kind and level of
// the tile elimination tree, all subdomains batched together.  Panel solves
// and trailing updates run on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Solve side: the interface operator F = sum_k B_k (K_rr^(k))^{-1}_{II} B_k^T
// + G S_c^{-1} G^T and the Dirichlet preconditioner sum_k B_k S_rIrI B_k^T
// (Section 2.1, Eqs. intProb and DirPrec) as batched dense GEMVs over the
// per-subdomain interface blocks with the signed Boolean gather fused in,
// followed by a deterministic two-term combine per multiplier row.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ieti {
namespace dev {

namespace {

constexpr int T = TILE;
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double pd2 __attribute__((ext_vector_type(2)));

// Value of lane `src` (wave-uniform) of a double, through two readlanes.
__device__ inline double readlane_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// A double moved across lanes by the DPP pattern CTRL (both halves alike).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 64 lanes of a wave (every lane active), result in every lane:
// pairs, quads, half-rows and rows of 16 through DPP moves inside the VALU
// (each step adds two values that every lane of the group sees in the same
// order up to commutation), then the four row sums through readlanes.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Sum over a 256-thread block, result valid in every thread (fixed order).
__device__ inline double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  const double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// Reduce a partials array of length n (small) in a fixed order by one block.
__device__ inline double reduce_partials(const double* part, int n, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  return block_sum256(v, red);
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// out[dst[i]] = val[i] (distinct destinations).
__global__ void k_scatter(double* out, const int64_t* dst, const double* val, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[dst[i]] = val[i];
}

// The tile pool from the assembled entries: one workgroup per tile; the
// tile is zeroed in LDS, its entries (one range of the destination-ordered
// list) placed there, and the tile written once in whole coalesced lines, in
// place of a fill of the whole pool followed by scattered 8-byte writes.  A
// tile without entries (fill of the factorisation) is written as zeros
// directly.
__global__ __launch_bounds__(256) void k_assemble_tiles(double* pool, const int64_t* dst, const double* val,
                                                        const int64_t* tile_ptr) {
  __shared__ __align__(16) double L[TILE * TILE];
  pd2* L2 = reinterpret_cast<pd2*>(L);
  constexpr int64_t TT = int64_t(TILE) * TILE;
  const int64_t t = blockIdx.x, base = t * TT;
  const int64_t p0 = tile_ptr[t], p1 = tile_ptr[t + 1];
  pd2* out = reinterpret_cast<pd2*>(pool + base);
  if (p0 == p1) {
#pragma unroll
    for (int s = 0; s < int(TT / 512); ++s) out[threadIdx.x + 256 * s] = pd2{0.0, 0.0};
    return;
  }
#pragma unroll
  for (int s = 0; s < int(TT / 512); ++s) L2[threadIdx.x + 256 * s] = pd2{0.0, 0.0};
  __syncthreads();
  for (int64_t i = p0 + threadIdx.x; i < p1; i += 256) L[dst[i] - base] = val[i];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < int(TT / 512); ++s) out[threadIdx.x + 256 * s] = L2[threadIdx.x + 256 * s];
}

// Cholesky of one 64x64 diagonal tile followed by the inverse of its lower
// factor, written to `inv`.  Four waves; lane i holds row i, wave w the 16
// columns 16w..16w+15 of it in registers.  Column k is finished by the wave
// that owns it and broadcast through LDS (two alternating buffers, so one
// barrier per column); every wave then updates its columns right of k with
// unconditional FMAs and selects, so the broadcast reads issue together.
// The inverse runs the same way column-oriented: lane c holds column c of
// L^{-1}, wave w its rows 16w..16w+15, reading column k of L from a
// transposed LDS copy and multiplying by the stored reciprocal pivots.  A
// pivot not above the subdomain's threshold piv_tol[sub] (a fixed fraction
// of the largest diagonal entry of its K_rr: numerically singular) records
// the subdomain (1-based) in err and continues with pivot 1.

__global__ __launch_bounds__(256) void k_potrf_inv(double* pool, double* inv, const int64_t* task,
                                                   const double* piv_tol, int* err) {
  __shared__ __align__(16) double Lt[T][T + 2];  // Lt[j][i] = L[i][j]; later X staging
  __shared__ __align__(16) double bc[2][T];
  __shared__ double dinv[T];
  const int64_t* tk = task + 3 * blockIdx.x;
  double* t = pool + tk[0];
  const int sub = int(tk[1]);
  const double tol = piv_tol[sub];
  double* tinv = inv + tk[2];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c0 = 16 * w;
  double a[16];
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) a[jj] = t[(c0 + jj) * T + lane];
  bool bad = false;
  // 64 column steps as 4 x 16: the inner steps are unrolled so that register
  // indices stay static, the outer loop is not (keeps the code in the
  // instruction cache)
#pragma unroll 1
  for (int kb = 0; kb < T; kb += 16)
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = kb + kk;
    double* col = bc[kk & 1];
    if (w == (kb >> 4)) {
      const double akk = readlane_f64(a[kk], k);
      const bool ok = akk > tol;
      bad = bad || !ok;
      // 1/sqrt(a) from the hardware estimate and two Newton steps
      // (y <- y (3 - a y^2) / 2), pivot sqrt(a) = a / sqrt(a): fewer dependent
      // instructions on the pivot's chain than an IEEE square root and division
      const double av = ok ? akk : 1.0;
      double rp = __builtin_amdgcn_rsq(av);
      rp = rp * (1.5 - 0.5 * av * rp * rp);
      rp = rp * (1.5 - 0.5 * av * rp * rp);
      const double piv = av * rp;
      const double lik = (lane == k) ? piv : (lane > k ? a[kk] * rp : 0.0);
      a[kk] = lik;
      col[lane] = lik;
      if (lane == 0) dinv[k] = rp;
    }
    __syncthreads();
    // trailing update of the wave's columns c0 + jj > k (wave-uniform cases)
    if (w >= (kb >> 4)) {
      const double li = col[lane];
      double cj[16];
#pragma unroll
      for (int jj = 0; jj < 16; jj += 2) {
        const double2 v = *reinterpret_cast<const double2*>(&col[c0 + jj]);
        cj[jj] = v.x;
        cj[jj + 1] = v.y;
      }
      if (w > (kb >> 4)) {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a[jj] -= li * cj[jj];
      } else {
#pragma unroll
        for (int jj = kk + 1; jj < 16; ++jj) a[jj] -= li * cj[jj];
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    const double v = (c0 + jj <= lane) ? a[jj] : 0.0;
    t[(c0 + jj) * T + lane] = v;
    Lt[c0 + jj][lane] = v;
  }
  __syncthreads();
  double x[16];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) x[rr] = (c0 + rr == lane) ? 1.0 : 0.0;
#pragma unroll 1
  for (int kb = 0; kb < T; kb += 16)
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = kb + kk;
    double* xk = bc[kk & 1];
    if (w == (kb >> 4)) {
      const double v = x[kk] * dinv[k];
      x[kk] = v;
      xk[lane] = v;
    }
    __syncthreads();
    if (w >= (kb >> 4)) {
      const double xv = xk[lane];
      double lk[16];
#pragma unroll
      for (int rr = 0; rr < 16; rr += 2) {
        const double2 v = *reinterpret_cast<const double2*>(&Lt[k][c0 + rr]);
        lk[rr] = v.x;
        lk[rr + 1] = v.y;
      }
      if (w > (kb >> 4)) {
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) x[rr] -= lk[rr] * xv;
      } else {
#pragma unroll
        for (int rr = kk + 1; rr < 16; ++rr) x[rr] -= lk[rr] * xv;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) Lt[lane][c0 + rr] = x[rr];  // Lt[c][r] = X[r][c]
  __syncthreads();
  for (int idx = threadIdx.x; idx < T * T; idx += 256) tinv[idx] = Lt[idx >> 6][idx & (T - 1)];
  if (bad && lane == 0) atomicMax(err, sub + 1);
}


// Accumulate A B^T (64x64 tiles, column-major) into the calling wave's
// 32x32 quadrant on the FP64 matrix cores.  Four waves, 2x2 blocks of 16x16
// accumulators each.  Operand layout of v_mfma_f64_16x16x4f64 (lane l):
//   A: row l%16, k l/16;  B: k l/16, col l%16;  accumulator element r:
//   row l/16 + 4r, col l%16 (checked on gfx950 with an in-bounds probe).
// The tiles pass through LDS one half of k at a time (columns 0..31 or
// 32..63 of a column-major tile: its two contiguous 16 KB halves); this
// accumulates one half.  Unrolled by two only: at four waves per SIMD the
// kernels using it have 128 VGPRs, and a full unroll hoists every LDS
// operand into registers and spills.
constexpr int KHALF = T * T / 2;

__device__ __attribute__((always_inline)) inline void mfma_khalf_lds(const double* As, const double* Bs, v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 2
  for (int kk = 0; kk < T / 8; ++kk) {
    const int k = 4 * kk + lk;
    const double a0 = As[k * T + 32 * wr + li];
    const double a1 = As[k * T + 32 * wr + 16 + li];
    const double b0 = Bs[k * T + 32 * wc + li];
    const double b1 = Bs[k * T + 32 * wc + 16 + li];
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
  }
}

// A 64x64 tile in LDS with columns padded to 65 entries: the MFMA layout's
// lanes run along columns 64 entries apart, which the padding spreads over
// the banks.  acc_to_lds writes the calling wave's accumulator quadrant
// there; lds_to_tile then writes the tile to global memory (C = L, or
// C = C - L) two entries of one column per thread and step, in whole
// coalesced lines, where direct stores from the MFMA layout write 32-byte
// pieces of 16 columns at once.
constexpr int LDT = T + 1;

__device__ __attribute__((always_inline)) inline void acc_to_lds(double* Ls, const v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1) + (lane >> 4), c0 = 32 * (w & 1) + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = r0 + 4 * r;
    Ls[c0 * LDT + rr] = acc[0][r];
    Ls[(c0 + 16) * LDT + rr] = acc[1][r];
    Ls[c0 * LDT + rr + 16] = acc[2][r];
    Ls[(c0 + 16) * LDT + rr + 16] = acc[3][r];
  }
}

template <bool SUB>
__device__ __attribute__((always_inline)) inline void lds_to_tile(double* C, const double* Ls) {
  pd2* C2 = reinterpret_cast<pd2*>(C);
#pragma unroll 2
  for (int s = 0; s < T * T / 512; ++s) {
    const int v = threadIdx.x + 256 * s, e = 2 * v;  // entries e, e + 1 of one column
    const double* l = Ls + (e >> 6) * LDT + (e & 63);
    pd2 c;
    if (SUB) {
      c = C2[v];
      c.x = c.x - l[0];
      c.y = c.y - l[1];
    } else {
      c.x = l[0];
      c.y = l[1];
    }
    C2[v] = c;
  }
}

// C -= sum_p A_p B_p^T over the pairs of one target tile (all its pending
// contributions), accumulated in registers and written once.  Each workgroup
// walks tasks b, b + gridDim.x, ... and their pairs as one sequence of
// stages, a stage being one half of k of one pair (columns 0..31 or 32..63 of
// both column-major tiles: their two contiguous 16 KB halves).  The stage's
// operands go through LDS (32 KB, in a 33 KB tile buffer that also carries
// the result out; four workgroups share a CU) while the next two stages load
// into registers: 256 KB of operands in flight per CU, twice what a
// one-pair-ahead pipeline with whole tiles in LDS (64 KB per workgroup, two
// per CU) keeps, which hides more of the memory latency behind the matrix
// cores.  Every target sums its pairs in order and k ascending, and leaves
// through LDS in whole lines (acc_to_lds, lds_to_tile).
struct UpdCursor {
  int64_t t, p0, np, q;
  int h;
};

__device__ __attribute__((always_inline)) inline void upd_skip_empty(UpdCursor& c, const int64_t* task, int64_t ntask,
                                                                     int64_t stride) {
  while (c.t < ntask && task[3 * c.t + 2] == 0) c.t += stride;
  if (c.t < ntask) {
    c.p0 = task[3 * c.t + 1];
    c.np = task[3 * c.t + 2];
  }
  c.q = 0;
  c.h = 0;
}

__device__ __attribute__((always_inline)) inline void upd_advance(UpdCursor& c, const int64_t* task, int64_t ntask,
                                                                  int64_t stride) {
  if (++c.h < 2) return;
  c.h = 0;
  if (++c.q < c.np) return;
  c.t += stride;
  upd_skip_empty(c, task, ntask, stride);
}

__device__ __attribute__((always_inline)) inline void upd_load_half(const double* pool, const int64_t* pair,
                                                                    const UpdCursor& c, pd2 r[8]) {
  const int64_t* pr = pair + 2 * (c.p0 + c.q);
  const pd2* A2 = reinterpret_cast<const pd2*>(pool + pr[0] + c.h * KHALF);
  const pd2* B2 = reinterpret_cast<const pd2*>(pool + pr[1] + c.h * KHALF);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    r[s] = A2[threadIdx.x + 256 * s];
    r[4 + s] = B2[threadIdx.x + 256 * s];
  }
}

__global__ __launch_bounds__(256, 4) void k_update_multi(double* pool, const int64_t* task, const int64_t* pair,
                                                        int64_t ntask) {
  // the stage's two half tiles; at a target's end the same LDS holds its
  // accumulated product (padded columns, acc_to_lds)
  __shared__ __align__(16) double Ls[T * LDT];
  double* As = Ls;
  double* Bs = Ls + KHALF;
  pd2* As2 = reinterpret_cast<pd2*>(As);
  pd2* Bs2 = reinterpret_cast<pd2*>(Bs);
  const int64_t stride = gridDim.x;
  UpdCursor cl;  // next stage to load
  cl.t = blockIdx.x;
  upd_skip_empty(cl, task, ntask, stride);
  if (cl.t >= ntask) return;
  UpdCursor cc = cl;  // stage whose operands the matrix cores consume next
  pd2 r0[8], r1[8];
  upd_load_half(pool, pair, cl, r0);
  upd_advance(cl, task, ntask, stride);
  if (cl.t < ntask) upd_load_half(pool, pair, cl, r1);
  upd_advance(cl, task, ntask, stride);
  v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  // one stage: its registers to LDS, the stage two ahead into the same
  // registers, the products, and the target's store after its last stage
  auto stage = [&](pd2 (&r)[8]) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      As2[threadIdx.x + 256 * s] = r[s];
      Bs2[threadIdx.x + 256 * s] = r[4 + s];
    }
    __syncthreads();
    if (cl.t < ntask) upd_load_half(pool, pair, cl, r);
    upd_advance(cl, task, ntask, stride);
    mfma_khalf_lds(As, Bs, acc);
    if (cc.h == 1 && cc.q + 1 == cc.np) {
      // C -= acc through LDS (whole coalesced lines of C)
      __syncthreads();
      acc_to_lds(Ls, acc);
      __syncthreads();
      lds_to_tile<true>(pool + task[3 * cc.t], Ls);
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = v4d{0, 0, 0, 0};
    }
    upd_advance(cc, task, ntask, stride);
  };
  while (true) {
    stage(r0);
    if (cc.t >= ntask) break;
    stage(r1);
    if (cc.t >= ntask) break;
  }
}

// Panel solve as a product with the inverted diagonal tile, X = A L_jj^{-T},
// one workgroup per tile: both operand tiles are loaded into registers at
// once and pass through LDS one half of k at a time (33 KB of LDS, so four
// workgroups share a CU and 256 KB of operands are in flight per CU, twice
// what whole tiles in LDS allow); X overwrites A through the same LDS in
// whole lines, with no second read of A.
__global__ __launch_bounds__(256, 4) void k_trsm_inv(double* pool, const double* inv, const int64_t* task) {
  __shared__ __align__(16) double Ls[T * LDT];  // the half tiles, then the product
  double* As = Ls;
  double* Bs = Ls + KHALF;
  pd2* As2 = reinterpret_cast<pd2*>(As);
  pd2* Bs2 = reinterpret_cast<pd2*>(Bs);
  const int64_t* tk = task + 2 * blockIdx.x;
  double* A = pool + tk[0];
  const pd2* A2 = reinterpret_cast<const pd2*>(A);
  const pd2* B2 = reinterpret_cast<const pd2*>(inv + tk[1]);
  pd2 ra[8], rb[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    ra[s] = A2[threadIdx.x + 256 * s];
    rb[s] = B2[threadIdx.x + 256 * s];
  }
  v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h) __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      As2[threadIdx.x + 256 * s] = ra[4 * h + s];
      Bs2[threadIdx.x + 256 * s] = rb[4 * h + s];
    }
    __syncthreads();
    mfma_khalf_lds(As, Bs, acc);
  }
  __syncthreads();
  acc_to_lds(Ls, acc);
  __syncthreads();
  lds_to_tile<false>(A, Ls);
}

// Copy (scaled) tiles into dense row-major blocks; optional mirrored copy;
// with dst32, the same entries rounded to FP32 into a second block of the
// same layout (the mixed-precision copies, written while the tile is in LDS).
// The tile is staged in LDS so that both the direct and the mirrored writes
// run along rows of the destination (consecutive threads, consecutive entries).
__global__ __launch_bounds__(256) void k_copy_tiles(const double* pool, const int64_t* task, double scale,
                                                    double* dst, float* dst32) {
  __shared__ double tl[T][T + 1];  // tl[b][a] = entry (a, b) of the tile
  const int64_t* tk = task + 5 * blockIdx.x;
  const double* t = pool + tk[0];
  const int64_t d0 = tk[1], dt = tk[2], ld = tk[3];
  const bool diag = tk[4] != 0;
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) tl[idx >> 6][idx & (T - 1)] = scale * t[idx];
  __syncthreads();
  // entry (a, b) to row a, column b: b runs along the threads
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
    const int a = idx >> 6, b = idx & (T - 1);
    if (!(diag && a < b)) {
      dst[d0 + a * ld + b] = tl[b][a];
      if (dst32) dst32[d0 + a * ld + b] = float(tl[b][a]);
    }
  }
  // entry (a, b) to row b, column a of the mirror: a runs along the threads
  if (dt >= 0)
    for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
      const int b = idx >> 6, a = idx & (T - 1);
      if (!(diag && a <= b)) {
        dst[dt + b * ld + a] = tl[b][a];
        if (dst32) dst32[dt + b * ld + a] = float(tl[b][a]);
      }
    }
}

// Triangular-solve tiles are read straight into registers: lane l of wave q
// loads entries l + 64 (16 q + k), k < 16, of a column-major 64x64 tile, i.e.
// 16 coalesced 512-byte column segments per wave; the wave index is made
// uniform so that the per-pair offsets and (forward) the 16 x values come
// through scalar loads.
//   forward (y -= L x):    lane = tile row a, the wave owns columns 16q..16q+15;
//                          per-lane partial sum over those columns, waves
//                          combined in LDS in fixed order.
//   transposed (y -= L^T x): lane = tile row b (x[b] per lane), the wave owns
//                          output entries a = 16q + k; per-lane products summed
//                          over the 64 lanes through LDS in fixed order.
constexpr int TRSV_CHUNK = 4;  // pairs whose tiles are in flight together

template <bool TR>
__device__ inline void trsv_tile_accumulate(const double* __restrict__ Lg, const double* __restrict__ xs, int lane,
                                            int q, double& accf, double (&acct)[16]) {
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = Lg[lane + 64 * (16 * q + k)];
  if (!TR) {
#pragma unroll
    for (int k = 0; k < 16; ++k) accf += v[k] * xs[16 * q + k];
  } else {
    const double xb = xs[lane];
#pragma unroll
    for (int k = 0; k < 16; ++k) acct[k] += v[k] * xb;
  }
}

// Combine the per-thread partials into the 64 entries of the target vector:
// out[a] = (forward) sum over waves of accf, (transposed) sum over lanes of acct.
template <bool TR>
__device__ inline double trsv_combine(double accf, const double (&acct)[16], int lane, int q, double* red) {
  if (!TR) {
    red[q * 64 + lane] = accf;
    __syncthreads();
    return (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
  }
  // red: 64 outputs x 65 (padded) lane partials
#pragma unroll
  for (int k = 0; k < 16; ++k) red[(16 * q + k) * 65 + lane] = acct[k];
  __syncthreads();
  // thread t: output a = t & 63, lanes 16 (t >> 6) .. +15
  const int a = threadIdx.x & 63, part = threadIdx.x >> 6;
  double sum = 0.0;
#pragma unroll
  for (int b = 0; b < 16; ++b) sum += red[a * 65 + 16 * part + b];
  __syncthreads();
  red[part * 64 + a] = sum;
  __syncthreads();
  return (red[a] + red[64 + a]) + (red[128 + a] + red[192 + a]);
}

// y_j <- L_jj^{-1} y_j (or L_jj^{-T} y_j) with the inverted diagonal tile.
template <bool TR>
__global__ __launch_bounds__(256) void k_trsv_diag_inv(const double* inv, const int64_t* task, double* y) {
  __shared__ double red[64 * 65];
  const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double* Lg = inv + task[2 * blockIdx.x];
  double* yv = y + task[2 * blockIdx.x + 1];
  double accf = 0.0, acct[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acct[k] = 0.0;
  trsv_tile_accumulate<TR>(Lg, yv, lane, q, accf, acct);
  const double out = trsv_combine<TR>(accf, acct, lane, q, red);
  if (threadIdx.x < 64) yv[threadIdx.x] = out;
}

// y_dst -= sum_p L_p x_p (forward) or sum_p L_p^T x_p (transposed) over the
// pairs [tile, vec_src] of one target, TRSV_CHUNK pairs in flight.
template <bool TR>
__global__ __launch_bounds__(256) void k_trsv_update_multi(const double* pool, const int64_t* task,
                                                           const int64_t* pair, double* y) {
  __shared__ double red[64 * 65];
  const int64_t* tk = task + 3 * blockIdx.x;
  double* yd = y + tk[0];
  const int64_t p0 = tk[1], np = tk[2];
  const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double accf = 0.0, acct[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acct[k] = 0.0;
  int64_t pp = 0;
  for (; pp + TRSV_CHUNK <= np; pp += TRSV_CHUNK) {
    double v[TRSV_CHUNK][16];
    const double* xs[TRSV_CHUNK];
#pragma unroll
    for (int c = 0; c < TRSV_CHUNK; ++c) {
      const double* Lg = pool + pair[2 * (p0 + pp + c)];
      xs[c] = y + pair[2 * (p0 + pp + c) + 1];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[c][k] = Lg[lane + 64 * (16 * q + k)];
    }
#pragma unroll
    for (int c = 0; c < TRSV_CHUNK; ++c) {
      if (!TR) {
#pragma unroll
        for (int k = 0; k < 16; ++k) accf += v[c][k] * xs[c][16 * q + k];
      } else {
        const double xb = xs[c][lane];
#pragma unroll
        for (int k = 0; k < 16; ++k) acct[k] += v[c][k] * xb;
      }
    }
  }
  for (; pp < np; ++pp)
    trsv_tile_accumulate<TR>(pool + pair[2 * (p0 + pp)], y + pair[2 * (p0 + pp) + 1], lane, q, accf, acct);
  const double out = trsv_combine<TR>(accf, acct, lane, q, red);
  if (threadIdx.x < 64) yd[threadIdx.x] -= out;
}

__global__ void k_sum_sources(const double* src, const int64_t* ptr, const int64_t* idx, int64_t nout, double* out) {
  const int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int64_t q = ptr[o]; q < ptr[o + 1]; ++q) s += src[idx[q]];
  out[o] = s;
}

// Problems of a batch: descriptor pd[PD_N * p + field] (see kernels.hpp);
// row blocks blk[2 b] = first multiplier row, blk[2 b + 1] = problem, each
// block holding at most 256 rows of one problem.
__device__ inline int64_t blk_rows(const int64_t* blk, const int64_t* pd, int64_t b, int64_t* row0) {
  *row0 = blk[2 * b];
  const int64_t mr1 = pd[PD_N * blk[2 * b + 1] + PD_MR1];
  return (mr1 - *row0) < 256 ? (mr1 - *row0) : 256;
}

// G_p[row][c] = sum over the row's two subdomains of +-Phi[slot][local primal of c]
// (thread per multiplier row, rows of one problem per block)
__global__ void k_build_G(const double* Phi, const int64_t* row_src, const int64_t* slot_phi_row,
                          const int32_t* I_sub, const int32_t* g2l, const int64_t* g2l_off, double* G,
                          const int64_t* pd, const int64_t* blk) {
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, blockIdx.x, &row0);
  if (int64_t(threadIdx.x) >= nrow) return;
  const int64_t* P = pd + PD_N * blk[2 * blockIdx.x + 1];
  const int64_t row = row0 + threadIdx.x, n_gp = P[PD_NGP];
  double* Gr = G + P[PD_H] + (row - P[PD_MR0]) * n_gp;
  for (int64_t c = 0; c < n_gp; ++c) {
    double g = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int64_t slot = row_src[2 * row + side];
      const int k = I_sub[slot];
      const int loc = g2l[g2l_off[k] + c];
      if (loc >= 0) g += (side == 0 ? 1.0 : -1.0) * Phi[slot_phi_row[slot] + loc];
    }
    Gr[c] = g;
  }
}

// ---- coarse problem as a tile factorisation (see CoarsePlan in the host plan)
//
// Tile fill: task [off_tile, source (0: S, 1: G, -1: none), source offset, ld,
// rows, cols, identity]; entry (a, b) of the column-major tile is
// source[off + a ld + b] for a < rows, b < cols, else 1 on the diagonal of an
// identity tile and 0.  Rows of the source are read along the threads and
// turned into tile columns through LDS.
__global__ __launch_bounds__(256) void k_dense_to_tiles(double* pool, const int64_t* task, const double* S,
                                                        const double* G) {
  __shared__ double tl[T][T + 1];  // tl[a][b] = entry (a, b)
  const int64_t* tk = task + 7 * blockIdx.x;
  double* t = pool + tk[0];
  const int64_t sel = tk[1], off = tk[2], ld = tk[3], rows = tk[4], cols = tk[5];
  const bool ident = tk[6] != 0;
  const double* src = sel == 0 ? S : (sel == 1 ? G : nullptr);
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
    const int a = idx >> 6, b = idx & (T - 1);
    double v = (ident && a == b) ? 1.0 : 0.0;
    if (src && a < rows && b < cols) v = src[off + a * ld + b];
    tl[a][b] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
    const int b = idx >> 6, a = idx & (T - 1);
    t[idx] = tl[a][b];
  }
}

// Tile extraction: task [off_tile, dst offset, transposed dst offset or -1,
// ld, transposed ld, rows, cols]; entry (a, b), a < rows, b < cols, goes to
// dst[off + a ld + b] and to dst_t[off_t + b ld_t + a].
__global__ __launch_bounds__(256) void k_tiles_to_dense(const double* pool, const int64_t* task, double* dst,
                                                        double* dst_t) {
  __shared__ double tl[T][T + 1];  // tl[b][a] = entry (a, b)
  const int64_t* tk = task + 7 * blockIdx.x;
  const double* t = pool + tk[0];
  const int64_t off = tk[1], off_t = tk[2], ld = tk[3], ldt = tk[4], rows = tk[5], cols = tk[6];
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) tl[idx >> 6][idx & (T - 1)] = t[idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
    const int a = idx >> 6, b = idx & (T - 1);
    if (a < rows && b < cols) dst[off + a * ld + b] = tl[b][a];
  }
  if (off_t >= 0 && dst_t)
    for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
      const int b = idx >> 6, a = idx & (T - 1);
      if (a < rows && b < cols) dst_t[off_t + b * ldt + a] = tl[b][a];
    }
}

// Triangular solves with the coarse factor through its explicit inverse
// U = L_c^{-T} (row-major n x n per problem, upper triangular), one
// workgroup per problem:
//   transposed = 0: out = L_c^{-1} in = U^T in, out[c] = sum_{i <= c} U[i][c] in[i]
//                   (a thread per output, rows of U read along the threads);
//   transposed = 1: out = L_c^{-T} in = U in,   out[i] = sum_{c >= i} U[i][c] in[c]
//                   (a wave per output, lanes along the row, fixed-order wave sum).
__global__ __launch_bounds__(256) void k_tri_small_inv(const double* U, const double* in, double* out,
                                                       int transposed, const int64_t* pd) {
  const int64_t* P = pd + PD_N * blockIdx.x;
  const int64_t n = P[PD_NGP], g0 = P[PD_GP0];
  if (n <= 0) return;
  const double* Up = U + P[PD_SPI];
  const double* x = in + g0;
  double* y = out + g0;
  if (!transposed) {
    for (int64_t c = threadIdx.x; c < n; c += 256) {
      double s0 = 0.0, s1 = 0.0;
      int64_t i = 0;
      for (; i + 1 <= c; i += 2) {
        s0 += Up[i * n + c] * x[i];
        s1 += Up[(i + 1) * n + c] * x[i + 1];
      }
      for (; i <= c; ++i) s0 += Up[i * n + c] * x[i];
      y[c] = s0 + s1;
    }
  } else {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t i = w; i < n; i += 4) {
      double s = 0.0;
      for (int64_t c = i + lane; c < n; c += 64) s += Up[i * n + c] * x[c];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) y[i] = s;
    }
  }
}

// Signed Boolean gather of a multiplier vector into interface slots:
// xg[slot(+1 side)] = x[row], xg[slot(-1 side)] = -x[row]  (xg = B^T x).
__global__ void k_gather_rows(const double* x, const int64_t* row_src, int64_t m_r, double* xg, const double* ds) {
  const int64_t row = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (row >= m_r) return;
  const double v = x[row];
  const int64_t s0 = row_src[2 * row], s1 = row_src[2 * row + 1];
  xg[s0] = ds ? ds[s0] * v : v;
  xg[s1] = ds ? -ds[s1] * v : -v;
}

// Batched dense GEMV over the per-subdomain interface blocks, v = M_k xg_k
// for every interface slot, plus one partial of sum_slot xg * v per block.
// task: [matrix row start, first slot of the rows, nrows, ld (= padded n_I),
// first slot of the subdomain].  The subdomain's slice of xg is staged in
// LDS; each wave owns RPW rows at a time and streams them with 16-byte
// loads, U vectors per lane in flight per row, optionally non-temporal (the
// blocks are read once per application and do not fit the caches).  Every
// variant sums each row in the same order, so results are identical; only
// the per-block partials of xg.v are grouped differently.

// 16-byte vectors of stored matrix entries (FP64: 2 entries, FP32: 4)
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
template <typename MT>
struct Vec16;
template <>
struct Vec16<double> {
  using T = nd2;
  static constexpr int N = 2;
  __device__ static inline double dot(const T& m, const double* x) { return m.x * x[0] + m.y * x[1]; }
};
template <>
struct Vec16<float> {
  using T = nf4;
  static constexpr int N = 4;
  __device__ static inline double dot(const T& m, const double* x) {
    return (double(m.x) * x[0] + double(m.y) * x[1]) + (double(m.z) * x[2] + double(m.w) * x[3]);
  }
};

// Matrix entries stored as MT (double or float), vector and accumulation in FP64.
template <typename MT, int RPW, int U, bool NT>
__global__ __launch_bounds__(256) void k_gemv(const MT* M, const int64_t* task, const double* xg, double* v,
                                              double* part, const int* done, const int32_t* task_prob) {
  if (done && done[task_prob[blockIdx.x]]) return;
  using V = Vec16<MT>;
  using T = typename V::T;
  extern __shared__ __align__(16) double xs[];
  __shared__ double red[4];
  const int64_t* tk = task + 5 * blockIdx.x;
  const int64_t mrow0 = tk[0], slot0 = tk[1], nrows = tk[2], ld = tk[3], xslot0 = tk[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  {
    const double2* src = reinterpret_cast<const double2*>(xg + xslot0);
    double2* dst = reinterpret_cast<double2*>(xs);
    for (int64_t j = threadIdx.x; j < ld / 2; j += 256) dst[j] = src[j];
  }
  __syncthreads();
  const int64_t nvec = ld / V::N;
  double dsum = 0.0;
  for (int64_t rb = w * RPW; rb < nrows; rb += 4 * RPW) {
    double acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
    for (int64_t j0 = lane; j0 < nvec; j0 += 64 * U) {
      T mv[U][RPW];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const int64_t j = j0 + 64 * u;
          if (j < nvec && rb + r < nrows) {
            const T* row = reinterpret_cast<const T*>(M + mrow0 + (rb + r) * ld);
            if constexpr (NT) mv[u][r] = __builtin_nontemporal_load(row + j);
            else mv[u][r] = row[j];
          } else {
            mv[u][r] = T(0);
          }
        }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + 64 * u;
        if (j < nvec) {
          const double* xv = xs + V::N * j;
#pragma unroll
          for (int r = 0; r < RPW; ++r) acc[r] += V::dot(mv[u][r], xv);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const double sres = wave_sum(acc[r]);
      if (lane == 0 && rb + r < nrows) {
        v[slot0 + rb + r] = sres;
        dsum += sres * xs[slot0 - xslot0 + rb + r];
      }
    }
  }
  if (lane == 0) red[w] = dsum;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Symmetric interface GEMV (S_rIrI and (K_rr^{-1})_II are symmetric): only
// the lower 64x64 tiles of a block are read, each once; the diagonal tile is
// stored whole.  task: [matrix offset of tile (I, t0), ld, ncols (64 per
// tile, <= SYM_TILES tiles of tile row I starting at tile column t0), first
// slot of tile row I, first slot of tile column t0, partial offset].  Row
// role: y_I += A_{I,t} x_t over the task's tiles (a row partial of 64).
// Column role: y_t += A_{I,t}^T x_I from the same loaded entries (a column
// partial of 64 per tile; the diagonal tile's is not used).  Lane l holds
// the columns N (l + 64 j) + e of its vectors for every row, so the column
// role needs no cross-lane sum; wave q takes rows 16q..16q+15, four at a
// time, and sums each row across the lanes (fixed butterfly order).
// Sums of R values (R a power of two, <= 64) over the 64 lanes of a wave at
// once: each butterfly step exchanges the half of the values a lane does not
// keep, so R values cost R - 1 + log2(64 / R) exchanges instead of 6 R.  On
// return lane l holds the total of value r = l >> (6 - log2 R) (fixed order).
template <int R>
__device__ inline double multi_wave_sum(double (&v)[R]) {
  const int lane = threadIdx.x & 63;
  int n = R, off = 32;
#pragma unroll
  for (; n > 1; n >>= 1, off >>= 1) {
    const bool hi = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
      const double send = hi ? v[i] : v[i + n / 2];
      const double keep = hi ? v[i + n / 2] : v[i];
      v[i] = keep + __shfl_xor(send, off, 64);
    }
  }
  double t = v[0];
#pragma unroll
  for (; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  return t;
}

template <typename MT>
__global__ __launch_bounds__(64 * SYM_WAVES, 2) void k_gemv_sym(const MT* M, const int64_t* task, const double* xg, double* part,
                                                  const int* done, const int32_t* task_prob) {
  const int64_t* tk = task + SYM_TASK * blockIdx.x;
  if (tk[2] == 0) return;  // empty record: a CU without a second task
  if (done && done[task_prob[blockIdx.x]]) return;
  using V = Vec16<MT>;
  using T = typename V::T;
  static_assert(SYM_TILES % V::N == 0, "a lane's 16-byte vectors must tile the task's columns exactly");
  constexpr int NJ = SYM_TILES * 64 / (64 * V::N);  // vectors per lane and row
  constexpr int RW = 64 / SYM_WAVES;                 // rows per wave
  constexpr int RB = 4 < RW ? 4 : RW;                // rows per batch (4 NJ vectors in flight per lane)
  __shared__ double rows[64];
  __shared__ double cred[SYM_WAVES][SYM_TILES * 64];
  const MT* A = M + tk[0];
  const int64_t ld = tk[1];
  const int ncols = int(tk[2]);
  const int nrows_in = int(tk[6]), ncols_in = int(tk[7]);  // inside n_I: the padding is not read
  const double* xr = xg + tk[3];
  const double* xc = xg + tk[4];
  const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double x[NJ][V::N], cacc[NJ][V::N];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int c0 = V::N * (lane + 64 * j);
#pragma unroll
    for (int e = 0; e < V::N; ++e) {
      x[j][e] = c0 < ncols_in ? xc[c0 + e] : 0.0;
      cacc[j][e] = 0.0;
    }
  }
  constexpr int SH = RB == 16 ? 2 : RB == 8 ? 3 : RB == 4 ? 4 : RB == 2 ? 5 : 6;  // lane >> SH = row of a batch
#pragma unroll 1
  for (int i = 0; i < RW; i += RB) {
    T mv[RB][NJ];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const T* row = reinterpret_cast<const T*>(A + (RW * q + i + r) * ld);
      const bool in = RW * q + i + r < nrows_in;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        mv[r][j] = in && V::N * (lane + 64 * j) < ncols_in ? __builtin_nontemporal_load(row + lane + 64 * j) : T(0);
    }
    double racc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double xa = xr[RW * q + i + r];
      double sacc = 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        sacc += V::dot(mv[r][j], x[j]);
#pragma unroll
        for (int e = 0; e < V::N; ++e) cacc[j][e] += double(mv[r][j][e]) * xa;
      }
      racc[r] = sacc;
    }
    // the batch's row sums: lane l ends with row l >> SH of the batch
    const double rsum = multi_wave_sum<RB>(racc);
    if ((lane & ((1 << SH) - 1)) == 0) rows[RW * q + i + (lane >> SH)] = rsum;
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < V::N; ++e) cred[q][V::N * (lane + 64 * j) + e] = cacc[j][e];
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += 64 * SYM_WAVES) {
    const int64_t dst = tk[8 + (c >> 6)];
    if (dst >= 0) {
      double sum = 0.0;
#pragma unroll
      for (int g = 0; g < SYM_WAVES; g += 2) sum += cred[g][c] + cred[g + 1][c];
      part[dst + (c & 63)] = sum;
    }
  }
  if (threadIdx.x < 64) part[tk[5] + threadIdx.x] = rows[threadIdx.x];
}

// t_p[c] = sum over the problem's row blocks b of part_t[b][c] for the 64
// columns c0..c0+63 of one problem (chunk task [problem, c0]): four thread
// groups split the blocks, combined in fixed order.  Once per iteration,
// before the operator's second half reads t.
__device__ inline void coarse_reduce_chunk(const double* part_t, const int64_t* pd, const int64_t* ctask,
                                           double* t, const int* done) {
  __shared__ double acc4[4][64];
  const int64_t pid = ctask[0], c0 = ctask[1];
  if (done && done[pid]) return;
  const int64_t* P = pd + PD_N * pid;
  const int64_t n_gp = P[PD_NGP], nb = P[PD_B1] - P[PD_B0];
  const double* pt = part_t + P[PD_PT];
  const int cl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t c = c0 + cl;
  double s0 = 0.0, s1 = 0.0;
  if (c < n_gp) {
    int64_t b = q;
    for (; b + 4 < nb; b += 8) {
      s0 += pt[b * n_gp + c];
      s1 += pt[(b + 4) * n_gp + c];
    }
    if (b < nb) s0 += pt[b * n_gp + c];
  }
  acc4[q][cl] = s0 + s1;
  __syncthreads();
  if (q == 0 && c < n_gp) t[P[PD_GP0] + c] = (acc4[0][cl] + acc4[1][cl]) + (acc4[2][cl] + acc4[3][cl]);
}

// Output block of 64 slots: v = sum of its contiguous partials (64 entries
// apiece), split into four groups (partials g, g + 4, ...) summed by the four
// waves and combined in fixed order; the block's dot partial
// part_g[b] = sum_slots xg v.  blk: [first slot, first partial, count].
__global__ __launch_bounds__(256) void k_gemv_sym_reduce(const double* part, const int64_t* blk, const double* xg,
                                                         double* v, double* part_g, const int* done,
                                                         const int32_t* blk_prob, int64_t nblk, const double* part_t,
                                                         const int64_t* pd, const int64_t* ctask, double* tvec) {
  // workgroups past the output blocks reduce the coarse partials (t = H^T p)
  if (int64_t(blockIdx.x) >= nblk) {
    coarse_reduce_chunk(part_t, pd, ctask + 2 * (blockIdx.x - nblk), tvec, done);
    return;
  }
  if (done && done[blk_prob[blockIdx.x]]) return;
  __shared__ double red[4][64];
  const int64_t* b = blk + 3 * blockIdx.x;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const double* p = part + b[1] + lane;
  const int n = int(b[2]);
  const int64_t slot = b[0] + lane;
  const double xs = g == 0 ? xg[slot] : 0.0;  // needed after the sum: loaded with the partials
  double s0 = 0.0, s1 = 0.0;
  int k = g;
  for (; k + 4 < n; k += 8) {
    s0 += p[64 * k];
    s1 += p[64 * (k + 4)];
  }
  if (k < n) s0 += p[64 * k];
  red[g][lane] = s0 + s1;
  __syncthreads();
  if (g == 0) {
    const double val = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    v[slot] = val;
    const double d = wave_sum(val * xs);
    if (lane == 0) part_g[blockIdx.x] = d;
  }
}

__global__ void k_to_float(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = float(in[i]);
}

// Sum of n partials by one block: the first 3072 are loaded all at once (12
// per thread, one memory round trip), any further ones in a loop; the result
// (fixed summation order) is returned to every thread.
__device__ inline double reduce_partials_fast(const double* part, int n, double* red) {
  double a[12];
#pragma unroll
  for (int u = 0; u < 12; ++u) {
    const int i = threadIdx.x + 256 * u;
    a[u] = i < n ? part[i] : 0.0;
  }
  double s = (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))) + ((a[8] + a[9]) + (a[10] + a[11]));
  for (int i = threadIdx.x + 3072; i < n; i += 256) s += part[i];
  return block_sum256(s, red);
}

__global__ __launch_bounds__(256) void k_coarse_reduce(const double* part_t, const int64_t* pd, const int64_t* ctask,
                                                       double* t, const int* done) {
  coarse_reduce_chunk(part_t, pd, ctask + 2 * blockIdx.x, t, done);
}

// out[c] = sum over the problem's rows of Ht_p[c][row] x[row] (block per global primal index)
__global__ __launch_bounds__(256) void k_coarse_project(const double* Ht, const double* x, double* out,
                                                        const int64_t* pd, const int32_t* cprob) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  const int64_t* P = pd + PD_N * cprob[c];
  const int64_t m = P[PD_MR1] - P[PD_MR0], cl = c - P[PD_GP0];
  const double* Hc = Ht + P[PD_HT] + cl * m;
  const double* xp = x + P[PD_MR0];
  double s = 0.0;
  for (int64_t row = threadIdx.x; row < m; row += 256) s += Hc[row] * xp[row];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[c] = s;
}

// sum_c H_p[row][c] t[c] for one row of problem P, read from the transposed
// copy Ht_p (n_gp x m): consecutive rows of a wave read consecutive entries
template <typename HT>
__device__ inline double coarse_row(const HT* Ht, const int64_t* P, int64_t row, const double* t) {
  const int64_t n_gp = P[PD_NGP], m = P[PD_MR1] - P[PD_MR0];
  const HT* Hc = Ht + P[PD_HT] + (row - P[PD_MR0]);
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  int64_t c = 0;
  for (; c + 3 < n_gp; c += 4) {
    c0 += double(Hc[c * m]) * t[c];
    c1 += double(Hc[(c + 1) * m]) * t[c + 1];
    c2 += double(Hc[(c + 2) * m]) * t[c + 2];
    c3 += double(Hc[(c + 3) * m]) * t[c + 3];
  }
  for (; c < n_gp; ++c) c0 += double(Hc[c * m]) * t[c];
  return (c0 + c1) + (c2 + c3);
}

// q[row] = v[+1 slot] - v[-1 slot] + sum_c H_p[row][c] t_p[c]  (H may be null)
__global__ __launch_bounds__(256) void k_combine(const double* v, const int64_t* row_src, const double* Ht,
                                                 const double* t, double* q, const int64_t* pd, const int64_t* blk,
                                                 const double* ds) {
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, blockIdx.x, &row0);
  if (int64_t(threadIdx.x) >= nrow) return;
  const int64_t* P = pd + PD_N * blk[2 * blockIdx.x + 1];
  const int64_t row = row0 + threadIdx.x;
  const int64_t s0 = row_src[2 * row], s1 = row_src[2 * row + 1];
  double val = ds ? ds[s0] * v[s0] - ds[s1] * v[s1] : v[s0] - v[s1];
  if (Ht && P[PD_NGP] > 0) val += coarse_row(Ht, P, row, t + P[PD_GP0]);
  q[row] = val;
}

// PCG, first half of an iteration (after v = Sinv_k B_k^T p), per problem p of
// the block: t = H_p^T p (reduced from pcg_M's block partials), p^T F p = sum xg.v + t.t
// over the problem's GEMV tasks, alpha = rz / p^T F p, q = B v + H t,
// lambda += alpha p, r -= alpha q, gather B^T r for the preconditioner,
// partials of ||r||^2.  scal + 8 p: [0..1] rz (ping-pong by parity),
// [2] alpha, [3] beta, [4] tol^2, [5] ||r||^2.  gt: GEMV task range index.
template <typename HT>
__global__ __launch_bounds__(256) void k_pcg_F(const double* v, const int64_t* row_src, const HT* Ht,
                                               const double* tvec, const double* part_g, const double* p,
                                               double* lam, double* r, double* xg_r, double* part_rr, double* scal,
                                               int par, int* done, int* err, const int64_t* pd, const int64_t* blk,
                                               int gt, const double* ds) {
  const int64_t b = blockIdx.x, pid = blk[2 * b + 1];
  if (done[pid]) return;
  extern __shared__ double tl[];
  __shared__ double red[4];
  const int64_t* P = pd + PD_N * pid;
  const int64_t n_gp = P[PD_NGP];
  // the row's operands do not depend on the reductions: their loads go first
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, b, &row0);
  const bool act = int64_t(threadIdx.x) < nrow;
  const int64_t row = row0 + threadIdx.x;
  int64_t s0 = 0, s1 = 0;
  double vd = 0.0, pr = 0.0, lr = 0.0, rv = 0.0;
  if (act) {
    s0 = row_src[2 * row];
    s1 = row_src[2 * row + 1];
    vd = v[s0] - v[s1];
    pr = p[row];
    lr = lam[row];
    rv = r[row];
  }
  // t = H_p^T p (reduced once per iteration by the coarse reduction) into LDS
  double tt = 0.0;
  for (int64_t c = threadIdx.x; c < n_gp; c += 256) {
    const double tc = tvec[P[PD_GP0] + c];
    tl[c] = tc;
    tt += tc * tc;
  }
  const double tt_all = block_sum256(tt, red);
  const double pq = reduce_partials_fast(part_g + P[PD_T0 + 2 * gt], int(P[PD_T0 + 2 * gt + 1] - P[PD_T0 + 2 * gt]),
                                         red) +
                    tt_all;
  double* sc = scal + 8 * pid;
  if (!(pq > 0.0)) {
    if (b == P[PD_B0] && threadIdx.x == 0) {
      *err = 1;
      done[pid] = 3;
    }
    return;
  }
  const double alpha = sc[par] / pq;
  double rr = 0.0;
  if (act) {
    double q = vd;
    if (n_gp > 0) q += coarse_row(Ht, P, row, tl);
    lam[row] = lr + alpha * pr;
    const double rn = rv - alpha * q;
    r[row] = rn;
    rr = rn * rn;
    xg_r[s0] = ds ? ds[s0] * rn : rn;
    xg_r[s1] = ds ? -ds[s1] * rn : -rn;
  }
  const double srr = block_sum256(rr, red);
  if (threadIdx.x == 0) part_rr[b] = srr;
  if (b == P[PD_B0] && threadIdx.x == 0) sc[2] = alpha;
}

// PCG, second half (after w = S_k B_k^T r), per problem p of the block:
// convergence test on ||r||^2, rz = sum xg_r.w, z = B w, beta = rz / rz_old,
// p = z + beta p, gather B^T p for the next operator GEMV and the block
// partials of H_p^T p.  init = 1 starts the recurrence (beta = 0, no test).
template <typename HT>
__global__ __launch_bounds__(256) void k_pcg_M(const double* w, const int64_t* row_src, const HT* H,
                                               const double* part_g, const double* part_rr, double* p, double* z,
                                               double* xg_p, double* part_t, double* scal, int par, int* done,
                                               int* iters, int init, const int64_t* pd, const int64_t* blk, int gt,
                                               const double* ds, double* hist, int hcap) {
  const int64_t b = blockIdx.x, pid = blk[2 * b + 1];
  if (done[pid]) return;
  __shared__ double red[4];
  __shared__ double pl[256];
  const int64_t* P = pd + PD_N * pid;
  double* sc = scal + 8 * pid;
  const bool first = b == P[PD_B0];
  // the row's operands do not depend on the reductions: their loads go first
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, b, &row0);
  const bool act = int64_t(threadIdx.x) < nrow;
  const int64_t row = row0 + threadIdx.x;
  int64_t s0 = 0, s1 = 0;
  double zz = 0.0, pold = 0.0;
  if (act) {
    s0 = row_src[2 * row];
    s1 = row_src[2 * row + 1];
    zz = ds ? ds[s0] * w[s0] - ds[s1] * w[s1] : w[s0] - w[s1];
    if (!init) pold = p[row];
  }
  const double rz = reduce_partials_fast(part_g + P[PD_T0 + 2 * gt], int(P[PD_T0 + 2 * gt + 1] - P[PD_T0 + 2 * gt]),
                                         red);
  if (!init) {
    const double rr = reduce_partials_fast(part_rr + P[PD_B0], int(P[PD_B1] - P[PD_B0]), red);
    if (first && threadIdx.x == 0) {
      const int it = iters[pid];
      iters[pid] = it + 1;
      sc[5] = rr;
      if (hist && it < hcap) hist[(pid * hcap + it) * 2] = sc[2];
    }
    if (rr <= sc[4]) {
      if (first && threadIdx.x == 0) done[pid] = 1;
      return;
    }
  }
  const double beta = init ? 0.0 : rz / sc[par];
  if (first && threadIdx.x == 0) {
    sc[init ? 0 : 1 - par] = rz;
    sc[3] = beta;
    if (hist && !init && iters[pid] - 1 < hcap) hist[(pid * hcap + iters[pid] - 1) * 2 + 1] = beta;
  }
  double pv = 0.0;
  if (act) {
    z[row] = zz;
    // the first direction is z itself: p holds no value yet (not even a finite one)
    pv = init ? zz : zz + beta * pold;
    p[row] = pv;
    xg_p[s0] = pv;
    xg_p[s1] = -pv;
  }
  pl[threadIdx.x] = pv;
  __syncthreads();
  // block partials of H_p^T p: 64 columns per pass, four row quarters per column
  __shared__ double acc4[4][64];
  const int64_t n_gp = P[PD_NGP];
  const HT* Hb = H + P[PD_H] + (row0 - P[PD_MR0]) * n_gp;
  double* pt = part_t + P[PD_PT] + (b - P[PD_B0]) * n_gp;
  const int c0 = threadIdx.x & 63, q = threadIdx.x >> 6;
  for (int64_t cb = 0; cb < n_gp; cb += 64) {
    const int64_t c = cb + c0;
    double s = 0.0;
    if (c < n_gp) {
      const int64_t i0 = 64 * q, i1 = (64 * q + 64) < nrow ? 64 * q + 64 : nrow;
#pragma unroll 8
      for (int64_t i = i0; i < i1; ++i) s += double(Hb[i * n_gp + c]) * pl[i];
    }
    acc4[q][c0] = s;
    __syncthreads();
    if (q == 0 && c < n_gp) pt[c] = (acc4[0][c0] + acc4[1][c0]) + (acc4[2][c0] + acc4[3][c0]);
    __syncthreads();
  }
}

__global__ void k_gather_add(const double* y, const int64_t* idx, double sgn, int64_t n, double* out) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) out[i] += sgn * y[idx[i]];
}

// e[row] = sum_k s_k (K_rr^{-1} j_r)_I = -(y[A(src0)] - y[A(src1)]) with y the forward solve.
__global__ void k_rhs_assemble(const double* y, const int64_t* A_aug, const int64_t* row_src, int64_t m_r, double* e) {
  const int64_t row = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (row >= m_r) return;
  e[row] = -(y[A_aug[row_src[2 * row]]] - y[A_aug[row_src[2 * row + 1]]]);
}

// Sources of the recovery's transposed update: the local primal values
// a_p = C_k p at every padded primal position (0 on padding) and the jump
// u = (B_r^T lambda)_I at every padded E_I position (0 on padding).
__global__ void k_recovery_sources(double* y, const int64_t* p_pos, const int64_t* p_glob, int64_t np,
                                   const double* pglob, const int64_t* A_aug, const int32_t* I_row,
                                   const double* I_sign, int64_t nslots, const double* lam) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < np) {
    const int64_t g = p_glob[i];
    y[p_pos[i]] = g >= 0 ? pglob[g] : 0.0;
  } else if (i < np + nslots) {
    const int64_t t = i - np;
    const int32_t row = I_row[t];
    y[A_aug[t]] = row >= 0 ? I_sign[t] * lam[row] : 0.0;
  }
}

__global__ void k_write_output(const double* y, const int64_t* src, const int64_t* edge, int64_t n, double* a) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) a[edge[i]] = y[src[i]];
}

__global__ void k_write_primal(const double* pglob, const int64_t* primal_edges, int64_t n_gp, double* a) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n_gp) a[primal_edges[i]] = pglob[i];
}

// b[row] = e[row] - sum_c H_p[row][c] w_p[c]
__global__ __launch_bounds__(256) void k_axpy_rows(const double* Ht, const double* w, const double* e, double* b,
                                                   const int64_t* pd, const int64_t* blk) {
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, blockIdx.x, &row0);
  if (int64_t(threadIdx.x) >= nrow) return;
  const int64_t* P = pd + PD_N * blk[2 * blockIdx.x + 1];
  const int64_t row = row0 + threadIdx.x;
  const double s = P[PD_NGP] > 0 ? coarse_row(Ht, P, row, w + P[PD_GP0]) : 0.0;
  b[row] = e[row] - s;
}

// part[b] = sum over the rows of block b of x y
__global__ __launch_bounds__(256) void k_dot_blocks(const double* x, const double* y, double* part, const int64_t* pd,
                                                    const int64_t* blk) {
  __shared__ double red[4];
  int64_t row0;
  const int64_t nrow = blk_rows(blk, pd, blockIdx.x, &row0);
  const int64_t row = row0 + threadIdx.x;
  const double v = int64_t(threadIdx.x) < nrow ? x[row] * y[row] : 0.0;
  const double sum = block_sum256(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

__global__ void k_axpby(const double* x, const double* y, double* out, double a, double b, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = a * x[i] + b * y[i];
}

__global__ void k_vec_copy(const double* x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = x[i];
}


int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return int(g);
}

}  // namespace

void fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void scatter(double* out, const int64_t* dst, const double* val, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, out, dst, val, n);
}
void assemble_tiles(double* pool, const int64_t* dst, const double* val, const int64_t* tile_ptr, int64_t ntile,
                    hipStream_t s) {
  if (ntile <= 0) return;
  hipLaunchKernelGGL(k_assemble_tiles, dim3(ntile), dim3(256), 0, s, pool, dst, val, tile_ptr);
}
void potrf_tiles(double* pool, double* inv, const int64_t* task, int64_t ntask, const double* piv_tol, int* err,
                 hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_potrf_inv, dim3(ntask), dim3(256), 0, s, pool, inv, task, piv_tol, err);
}
void trsm_tiles(double* pool, const double* inv, const int64_t* task, int64_t ntask, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_trsm_inv, dim3(ntask), dim3(256), 0, s, pool, inv, task);
}
void update_tiles(double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, hipStream_t s,
                  int64_t max_wgs) {
  if (ntask <= 0) return;
  const int64_t cap = max_wgs > 0 ? max_wgs : UPDATE_WGS;
  const int64_t nwg = ntask < cap ? ntask : cap;
  hipLaunchKernelGGL(k_update_multi, dim3(nwg), dim3(256), 0, s, pool, task, pair, ntask);
}
void copy_tiles(const double* pool, const int64_t* task, int64_t ntask, double scale, double* dst, hipStream_t s,
                float* dst32) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_copy_tiles, dim3(ntask), dim3(256), 0, s, pool, task, scale, dst, dst32);
}
void trsv_diag(const double* inv, const int64_t* task, int64_t ntask, double* y, bool transposed, hipStream_t s) {
  if (ntask <= 0) return;
  if (transposed)
    hipLaunchKernelGGL(k_trsv_diag_inv<true>, dim3(ntask), dim3(256), 0, s, inv, task, y);
  else
    hipLaunchKernelGGL(k_trsv_diag_inv<false>, dim3(ntask), dim3(256), 0, s, inv, task, y);
}
void trsv_update(const double* pool, const int64_t* task, const int64_t* pair, int64_t ntask, double* y,
                 bool transposed, hipStream_t s) {
  if (ntask <= 0) return;
  if (transposed)
    hipLaunchKernelGGL(k_trsv_update_multi<true>, dim3(ntask), dim3(256), 0, s, pool, task, pair, y);
  else
    hipLaunchKernelGGL(k_trsv_update_multi<false>, dim3(ntask), dim3(256), 0, s, pool, task, pair, y);
}
void sum_sources(const double* src, const int64_t* ptr, const int64_t* idx, int64_t nout, double* out, hipStream_t s) {
  if (nout <= 0) return;
  hipLaunchKernelGGL(k_sum_sources, dim3(grid_for(nout, 256)), dim3(256), 0, s, src, ptr, idx, nout, out);
}
void build_G(const double* Phi, const int64_t* row_src, const int64_t* slot_phi_row, const int32_t* I_sub,
             const int32_t* g2l, const int64_t* g2l_off, double* G, const Batch& B, hipStream_t s) {
  if (B.n_gp_total <= 0 || B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_build_G, dim3(B.n_blk), dim3(256), 0, s, Phi, row_src, slot_phi_row, I_sub, g2l, g2l_off, G,
                     B.pd, B.blk);
}
void dense_to_tiles(double* pool, const int64_t* task, int64_t ntask, const double* S, const double* G,
                    hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_dense_to_tiles, dim3(ntask), dim3(256), 0, s, pool, task, S, G);
}
void tiles_to_dense(const double* pool, const int64_t* task, int64_t ntask, double* dst, double* dst_t, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_tiles_to_dense, dim3(ntask), dim3(256), 0, s, pool, task, dst, dst_t);
}
void tri_small_inv(const double* U, const double* in, double* out, bool transposed, const Batch& B, hipStream_t s) {
  if (B.n_gp_total <= 0 || B.n_prob <= 0) return;
  hipLaunchKernelGGL(k_tri_small_inv, dim3(B.n_prob), dim3(256), 0, s, U, in, out, transposed ? 1 : 0, B.pd);
}
void gather_rows(const double* x, const int64_t* row_src, int64_t m_r, double* xg, hipStream_t s, const double* ds) {
  if (m_r <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((m_r + 255) / 256), dim3(256), 0, s, x, row_src, m_r, xg, ds);
}
GemvShape gemv_shape(int variant) {
  static const int rpw[3] = {2, 4, 8};
  if (variant < 0 || variant >= GEMV_VARIANTS) variant = GEMV_DEFAULT;
  return GemvShape{rpw[variant / 4], 1 + (variant / 2) % 2, variant % 2};
}

template <typename MT, int RPW, int U, bool NT>
void gemv_launch(const MT* M, const int64_t* task, int64_t ntask, size_t lds, const double* xg, double* v,
                 double* part, const int* done, const int32_t* tprob, hipStream_t s, hipEvent_t ev_start,
                 hipEvent_t ev_stop) {
  if (ev_start)
    hipExtLaunchKernelGGL((k_gemv<MT, RPW, U, NT>), dim3(ntask), dim3(256), lds, s, ev_start, ev_stop, 0, M, task,
                          xg, v, part, done, tprob);
  else
    hipLaunchKernelGGL((k_gemv<MT, RPW, U, NT>), dim3(ntask), dim3(256), lds, s, M, task, xg, v, part, done, tprob);
}

template <typename MT, int RPW>
void gemv_dispatch_u(int u, int nt, const MT* M, const int64_t* task, int64_t ntask, size_t lds, const double* xg,
                     double* v, double* part, const int* done, const int32_t* tp, hipStream_t s, hipEvent_t a,
                     hipEvent_t b) {
  if (u == 1 && !nt) gemv_launch<MT, RPW, 1, false>(M, task, ntask, lds, xg, v, part, done, tp, s, a, b);
  else if (u == 1) gemv_launch<MT, RPW, 1, true>(M, task, ntask, lds, xg, v, part, done, tp, s, a, b);
  else if (!nt) gemv_launch<MT, RPW, 2, false>(M, task, ntask, lds, xg, v, part, done, tp, s, a, b);
  else gemv_launch<MT, RPW, 2, true>(M, task, ntask, lds, xg, v, part, done, tp, s, a, b);
}

template <typename MT>
void gemv_impl(const MT* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
               double* part, const int* done, const int32_t* tp, hipStream_t s, int variant, hipEvent_t ev_start,
               hipEvent_t ev_stop) {
  if (ntask <= 0) return;
  if (!done) tp = nullptr;
  const size_t lds = size_t(max_ld) * sizeof(double);
  const GemvShape g = gemv_shape(variant);
  if (g.rpw == 2)
    gemv_dispatch_u<MT, 2>(g.unroll, g.nt, M, task, ntask, lds, xg, v, part, done, tp, s, ev_start, ev_stop);
  else if (g.rpw == 4)
    gemv_dispatch_u<MT, 4>(g.unroll, g.nt, M, task, ntask, lds, xg, v, part, done, tp, s, ev_start, ev_stop);
  else gemv_dispatch_u<MT, 8>(g.unroll, g.nt, M, task, ntask, lds, xg, v, part, done, tp, s, ev_start, ev_stop);
}
void gemv(const double* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
          double* part, const int* done, const int32_t* task_prob, hipStream_t s, int variant, hipEvent_t ev_start,
          hipEvent_t ev_stop) {
  gemv_impl(M, task, ntask, max_ld, xg, v, part, done, task_prob, s, variant, ev_start, ev_stop);
}
void gemv(const float* M, const int64_t* task, int64_t ntask, int64_t max_ld, const double* xg, double* v,
          double* part, const int* done, const int32_t* task_prob, hipStream_t s, int variant, hipEvent_t ev_start,
          hipEvent_t ev_stop) {
  gemv_impl(M, task, ntask, max_ld, xg, v, part, done, task_prob, s, variant, ev_start, ev_stop);
}
template <typename MT>
void gemv_sym_impl(const MT* M, const SymGemv& g, const double* xg, double* v, double* part_g, const int* done,
                   hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, const CoarseReduce* cr, const Batch* B) {
  if (g.ntask <= 0 || g.nblk <= 0) return;
  const int32_t* tp = done ? g.task_prob : nullptr;
  const int32_t* bp = done ? g.blk_prob : nullptr;
  // the events bracket the tile kernel (the streaming part); the block
  // reduction is a separate small launch
  if (ev_start)
    hipExtLaunchKernelGGL(k_gemv_sym<MT>, dim3(g.ntask), dim3(64 * SYM_WAVES), 0, s, ev_start, ev_stop, 0, M, g.task,
                          xg, g.part, done, tp);
  else
    hipLaunchKernelGGL(k_gemv_sym<MT>, dim3(g.ntask), dim3(64 * SYM_WAVES), 0, s, M, g.task, xg, g.part, done, tp);
  const int64_t nc = (cr && B) ? cr->ntask : 0;
  hipLaunchKernelGGL(k_gemv_sym_reduce, dim3(g.nblk + nc), dim3(256), 0, s, g.part, g.blk, xg, v, part_g, done, bp,
                     g.nblk, nc ? cr->part_t : nullptr, nc ? B->pd : nullptr, nc ? cr->task : nullptr,
                     nc ? cr->t : nullptr);
}
void gemv_sym(const double* M, const SymGemv& g, const double* xg, double* v, double* part_g, const int* done,
              hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, const CoarseReduce* cr, const Batch* B) {
  gemv_sym_impl(M, g, xg, v, part_g, done, s, ev_start, ev_stop, cr, B);
}
void gemv_sym(const float* M, const SymGemv& g, const double* xg, double* v, double* part_g, const int* done,
              hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, const CoarseReduce* cr, const Batch* B) {
  gemv_sym_impl(M, g, xg, v, part_g, done, s, ev_start, ev_stop, cr, B);
}
void coarse_reduce(const CoarseReduce& c, const int* done, const Batch& B, hipStream_t s) {
  if (c.ntask <= 0) return;
  hipLaunchKernelGGL(k_coarse_reduce, dim3(c.ntask), dim3(256), 0, s, c.part_t, B.pd, c.task, c.t, done);
}
void to_float(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_float, dim3(grid_for(n, 256)), dim3(256), 0, s, in, out, n);
}
void coarse_project(const double* Ht, const double* x, double* out, const int32_t* cprob, const Batch& B,
                    hipStream_t s) {
  if (B.n_gp_total <= 0) return;
  hipLaunchKernelGGL(k_coarse_project, dim3(B.n_gp_total), dim3(256), 0, s, Ht, x, out, B.pd, cprob);
}
void combine(const double* v, const int64_t* row_src, const double* H, const double* t, double* q, const Batch& B,
             hipStream_t s, const double* ds) {
  if (B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_combine, dim3(B.n_blk), dim3(256), 0, s, v, row_src, H, t, q, B.pd, B.blk, ds);
}
template <typename HT>
void pcg_F_impl(const double* v, const int64_t* row_src, const HT* Ht, const double* tvec, const double* part_g,
                const double* p, double* lam, double* r, double* xg_r, double* part_rr, double* scal, int par, int* done,
                int* err, const Batch& B, int gt, hipStream_t s, const double* ds) {
  if (B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_pcg_F<HT>, dim3(B.n_blk), dim3(256), size_t(B.max_gp > 0 ? B.max_gp : 1) * sizeof(double), s,
                     v, row_src, Ht, tvec, part_g, p, lam, r, xg_r, part_rr, scal, par, done, err, B.pd, B.blk, gt, ds);
}
void pcg_F(const double* v, const int64_t* row_src, const double* Ht, const double* tvec, const double* part_g,
           const double* p, double* lam, double* r, double* xg_r, double* part_rr, double* scal, int par, int* done,
           int* err, const Batch& B, int gt, hipStream_t s, const double* ds) {
  pcg_F_impl(v, row_src, Ht, tvec, part_g, p, lam, r, xg_r, part_rr, scal, par, done, err, B, gt, s, ds);
}
void pcg_F(const double* v, const int64_t* row_src, const float* Ht, const double* tvec, const double* part_g,
           const double* p, double* lam, double* r, double* xg_r, double* part_rr, double* scal, int par, int* done,
           int* err, const Batch& B, int gt, hipStream_t s, const double* ds) {
  pcg_F_impl(v, row_src, Ht, tvec, part_g, p, lam, r, xg_r, part_rr, scal, par, done, err, B, gt, s, ds);
}
template <typename HT>
void pcg_M_impl(const double* w, const int64_t* row_src, const HT* H, const double* part_g, const double* part_rr,
                double* p, double* z, double* xg_p, double* part_t, double* scal, int par, int* done, int* iters,
                int init, const Batch& B, int gt, hipStream_t s, const double* ds) {
  if (B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_pcg_M<HT>, dim3(B.n_blk), dim3(256), 0, s, w, row_src, H, part_g, part_rr, p, z, xg_p, part_t,
                     scal, par, done, iters, init, B.pd, B.blk, gt, ds, B.hist, B.hcap);
}
void pcg_M(const double* w, const int64_t* row_src, const double* H, const double* part_g, const double* part_rr,
           double* p, double* z, double* xg_p, double* part_t, double* scal, int par, int* done, int* iters, int init,
           const Batch& B, int gt, hipStream_t s, const double* ds) {
  pcg_M_impl(w, row_src, H, part_g, part_rr, p, z, xg_p, part_t, scal, par, done, iters, init, B, gt, s, ds);
}
void pcg_M(const double* w, const int64_t* row_src, const float* H, const double* part_g, const double* part_rr,
           double* p, double* z, double* xg_p, double* part_t, double* scal, int par, int* done, int* iters, int init,
           const Batch& B, int gt, hipStream_t s, const double* ds) {
  pcg_M_impl(w, row_src, H, part_g, part_rr, p, z, xg_p, part_t, scal, par, done, iters, init, B, gt, s, ds);
}
void gather_add(const double* y, const int64_t* idx, double sgn, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_add, dim3((n + 255) / 256), dim3(256), 0, s, y, idx, sgn, n, out);
}
void rhs_assemble(const double* y, const int64_t* A_aug, const int64_t* row_src, int64_t m_r, double* e, hipStream_t s) {
  if (m_r <= 0) return;
  hipLaunchKernelGGL(k_rhs_assemble, dim3((m_r + 255) / 256), dim3(256), 0, s, y, A_aug, row_src, m_r, e);
}
void recovery_sources(double* y, const int64_t* p_pos, const int64_t* p_glob, int64_t np, const double* pglob,
                      const int64_t* A_aug, const int32_t* I_row, const double* I_sign, int64_t nslots,
                      const double* lam, hipStream_t s) {
  const int64_t n = np + nslots;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_recovery_sources, dim3(grid_for(n, 256)), dim3(256), 0, s, y, p_pos, p_glob, np, pglob, A_aug,
                     I_row, I_sign, nslots, lam);
}
void write_output(const double* y, const int64_t* src, const int64_t* edge, int64_t n, const double* pglob,
                  const int64_t* primal_edges, int64_t n_gp, double* a, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_write_output, dim3((n + 255) / 256), dim3(256), 0, s, y, src, edge, n, a);
  if (n_gp > 0)
    hipLaunchKernelGGL(k_write_primal, dim3((n_gp + 255) / 256), dim3(256), 0, s, pglob, primal_edges, n_gp, a);
}
void axpy_rows(const double* H, const double* w, const double* e, double* b, const Batch& B, hipStream_t s) {
  if (B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_axpy_rows, dim3(B.n_blk), dim3(256), 0, s, H, w, e, b, B.pd, B.blk);
}
void axpby(const double* x, const double* y, double* out, double a, double b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, out, a, b, n);
}
void vec_copy(const double* x, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_vec_copy, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
}
void dot_blocks(const double* x, const double* y, double* part, const Batch& B, hipStream_t s) {
  if (B.n_blk <= 0) return;
  hipLaunchKernelGGL(k_dot_blocks, dim3(B.n_blk), dim3(256), 0, s, x, y, part, B.pd, B.blk);
}

}  // namespace dev
}  // namespace ieti
