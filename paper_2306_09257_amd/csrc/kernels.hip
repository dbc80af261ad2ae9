// HIP kernels of the APF library for gfx950 (MI355X).
//
// Every front of one elimination-tree level is processed by one launch of
// each kernel below; the host plan holds the per-level task arrays.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "apf_internal.h"
#include "kernels.h"

namespace apf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cinv(double2 a) {
  // 1/a = conj(a) / |a|^2, with a scaled by the power of two 2^-e of its
  // larger part (exact, and |a|^2 then neither overflows nor underflows):
  // one division instead of one per part and scale
  const double s = fmax(fabs(a.x), fabs(a.y));
  if (s == 0.0) return make_double2(0.0, 0.0);
  int e;
  (void)frexp(s, &e);
  const double ar = ldexp(a.x, -e), ai = ldexp(a.y, -e);
  const double t = 1.0 / (ar * ar + ai * ai);
  return make_double2(ldexp(ar * t, -e), ldexp(-ai * t, -e));
}
// by-value select: a conditional over lvalues would take the operands'
// addresses and push register arrays into scratch
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
__device__ __forceinline__ double2 ld2(const cplx *p) { return *reinterpret_cast<const double2 *>(p); }
// the same memory seen through the global address space (global_load
// instead of flat_load)
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const dvec2 gcplx;
__device__ __forceinline__ gcplx *as_global(const cplx *p) { return (gcplx *)p; }
__device__ __forceinline__ double2 ldg(gcplx *p) {
  const dvec2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(cplx *p, double2 v) { *reinterpret_cast<double2 *>(p) = v; }
// 16 bytes per lane straight from global memory into LDS: lane l's entry
// lands at dst + l (dst must be the same for the whole wave)
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;
__device__ __forceinline__ void ld_lds16(const cplx *src, double2 *dst) {
  __builtin_amdgcn_global_load_lds((glb_void *)src, (lds_void *)dst, 16, 0, 0);
}

// ---------------------------------------------------------------------------
// Zero the frontal workspaces of one level.
// ---------------------------------------------------------------------------
// One block per range; the host splits ranges into chunks of at most
// ZERO_CHUNK elements so that blocks are evenly loaded.
__global__ void k_zero(const ZeroRange *r) {
  const ZeroRange z = r[blockIdx.x];
  double2 *p = reinterpret_cast<double2 *>(z.ptr);
  for (int64_t i = threadIdx.x; i < z.n; i += blockDim.x) p[i] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Assembly of A (the 5-point UPML operator) into frontal cores, and of the
// source / projection rows into the channel panels.
// ---------------------------------------------------------------------------
__device__ double2 stretch(const Phys &P, double y) {
  // s(d) = 1 + i alpha (d/L)^m past the PML's inner face (half-row)
  double yt = P.npml_top - 0.5, yb = P.ny - P.npml_bot - 0.5;
  if (P.npml_top > 0 && y < yt) {
    double t = (yt - y) / P.npml_top;
    return make_double2(1.0, P.alpha_top * pow(t, (double)P.pml_power));
  }
  if (P.npml_bot > 0 && y > yb) {
    double t = (y - yb) / P.npml_bot;
    return make_double2(1.0, P.alpha_bot * pow(t, (double)P.pml_power));
  }
  return make_double2(1.0, 0.0);
}

// Stencil values of A for every node (a1): Aval[node][dir], dir 0 centre,
// 1 x-1, 2 x+1, 3 y-1, 4 y+1 (x periodic; entries beyond the first and last
// rows are never scattered).  A zero or non-finite permittivity sets
// ST_BAD_EPS in *status (the factorization reports it).
__global__ void k_stencil(Phys P, const double *eps, cplx *Aval, int *status) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= (int64_t)P.nx * P.ny) return;
  const int j = (int)(n / P.nx);
  const double2 sj = stretch(P, (double)j);
  const double2 up = cinv(stretch(P, j - 0.5)), dn = cinv(stretch(P, j + 0.5));
  const double ep = eps[n];
  if (!(fabs(ep) > 0.0) || !(fabs(ep) < INFINITY)) atomicOr(status, ST_BAD_EPS);
  double2 c = cadd(make_double2(2.0 * sj.x, 2.0 * sj.y), cadd(up, dn));
  c = csub(c, make_double2(P.h2 * ep * sj.x, P.h2 * ep * sj.y));
  cplx *o = Aval + n * 5;
  st2(o + 0, c);
  st2(o + 1, make_double2(-sj.x, -sj.y));
  st2(o + 2, make_double2(-sj.x, -sj.y));
  st2(o + 3, make_double2(-up.x, -up.y));
  st2(o + 4, make_double2(-dn.x, -dn.y));
}

// Scatter of the stencil values of one level's fronts into their cores.
__global__ void k_scatter_A(const AsmEntry *e, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const AsmEntry E = e[t];
  st2(E.dest, cadd(ld2(E.dest), ld2(E.src)));
}

__global__ void k_fill_int(int *p, int v) { *p = v; }

// Channel value at column i of order a in a medium: sqrt(sin q) phi_a(i), with
// q from sin^2(q/2) = h^2 eps/4 - sin^2(pi a/nx) and phi_a(i) = e^{2 pi i a i/nx}/sqrt(nx).
// channel_amp is the order's factor sqrt(sin q / nx), channel_phase the
// node's e^{+-2 pi i a i/nx}, with a i reduced mod nx exactly in FP64 (an
// integer below 2^53: the quotient's floor is off by at most one, and the
// products and differences are exact).
__device__ double channel_amp(const Phys &P, int a, double eps_medium) {
  double sa = sin(M_PI * (double)a / P.nx);
  double rhs = P.h2 * eps_medium * 0.25 - sa * sa;
  double q = 2.0 * asin(sqrt(rhs));
  return sqrt(sin(q) / P.nx);
}
__device__ double2 channel_phase(const Phys &P, int a, int i, bool conj_phase) {
  const double nx = (double)P.nx, x = (double)a * (double)i;
  double ph = x - floor(x / nx) * nx;
  if (ph < 0.0) ph += nx;
  else if (ph >= nx) ph -= nx;
  double ang = 2.0 * M_PI * ph / P.nx;
  double s, c;
  sincos(ang, &s, &c);
  return make_double2(c, conj_phase ? -s : s);
}
__device__ double2 channel_value(const Phys &P, int a, int i, double eps_medium, bool conj_phase) {
  const double amp = channel_amp(P, a, eps_medium);
  const double2 e = channel_phase(P, a, i, conj_phase);
  return make_double2(amp * e.x, amp * e.y);
}

// The orders' factors channel_amp of both panels (one thread per order).
__global__ void k_channel_amp(const ChanParams *cp, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const ChanParams &C = cp[t < cp[0].m ? 0 : 1];
  const int a = t < cp[0].m ? t : t - cp[0].m;
  C.amp[a] = channel_amp(C.P, C.orders[a], C.is_source ? C.P.eps_src : C.P.eps_prj);
}

// B rows: -2i sqrt(sin q_a) phi_a(i); C^T rows: sqrt(sin q_b) conj(phi_b(i)).
// Each row is stored whole: the assembly is the first writer of its rows.
__global__ void k_assemble_panel(const PanelEntry *e) {
  const PanelEntry E = e[blockIdx.x];
  const ChanParams &cp = *E.cp;
  const Phys &P = cp.P;
  const int is_source = cp.is_source, m = cp.m;
  const int i = E.node % P.nx;
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    // (the order's factor from the table channel_amp filled for the plan)
    const double amp = cp.amp[a];
    const double2 e = channel_phase(P, cp.orders[a], i, !is_source);
    double2 v = make_double2(amp * e.x, amp * e.y);
    if (is_source) v = make_double2(2.0 * v.y, -2.0 * v.x);   // times -2i
    st2(E.dest + a, v);
  }
}

// ---------------------------------------------------------------------------
// Pivot-block factorization: F11 = P L U with partial (row) pivoting, then the
// explicit inverses of the unit lower factor L and the upper factor U.  Output
// `tri` (p x p, rows in elimination-step order): strict lower part = L^-1
// (unit diagonal implied), upper part = U^-1; `perm[k]` = the row of F11 that
// step k pivoted on, so F11^-1 = U^-1 L^-1 P^T with (P^T X)[k] = X[perm[k]].
// The products of the factorization apply the two inverses in sequence;
// forming F11^-1 itself is avoided (it loses accuracy on nearly singular
// pivot blocks, which the Helmholtz operator produces when an eliminated
// subdomain is close to resonance).
//
// Phase A (LU): step k takes the largest not-yet-used row r of column k;
// rows do not move: every unused row x gets l_x = a[x][k]/a[r][k] stored in
// column k and a[x][j] -= l_x a[r][j] for j > k.
// Phase B (inverses): in-place Gauss-Jordan on L (unit, step order) and on U
// at once; step k updates the L triangle (i > k, j < k) with column k of L
// and row k of L, and the U triangle (i < k, j > k) with column k of U and
// row k of U scaled by 1/u_kk; the two touch disjoint entries.
//
// Symmetric mode (sym != 0; A = A^T, Sec. 2, so every pivot block is complex
// symmetric): only the lower triangle of the block is read (entry (i, j) with
// i < j taken from (j, i)) and step k pivots on row k, so F11 = L U with
// U = D L^T, the L D L^T factorization of the block, and perm is the identity.
// ---------------------------------------------------------------------------
constexpr int INV_MAXP = 1024;   // "no step" marker of a register row past p

// Register-blocked variant for p <= TR*RR = TC*RC: thread (ti, tj) of a
// TR x TC grid keeps entries (ti + TR*ra, tj + TC*ca) in registers.  Steps
// run as k = kq*TC + kc with kq unrolled, so the pivot column k is register
// column kq (a compile-time index) in the threads with tj == kc; only the
// pivot row, found at run time, needs a run-time register choice.
template <int TR, int TC, int RR, int RC>
__global__ __launch_bounds__(TR *TC) void k_lu_inv_reg(const FrontDev *fr, const int32_t *ids, int *status,
                                                       double *pivq, int sym) {
  constexpr int MAXP = TR * RR;
  static_assert(TR * RR == TC * RC, "square coverage");
  static_assert(MAXP < INV_MAXP, "the no-step marker must exceed every step");
  static_assert(TR <= 64 && (64 % TR) == 0, "a pivot-column group must sit inside one wave");
  const FrontDev F = fr[ids[blockIdx.x]];
  const int p = F.p, n = F.p + F.b;
  const int tid = threadIdx.x, ti = tid % TR, tj = tid / TR;
  __shared__ double2 rowbuf[MAXP], colbuf[MAXP];
  __shared__ int piv_row[MAXP], piv_step[MAXP];
  __shared__ int s_r, s_bad;
  __shared__ double s_pmin[TC], s_pmax[TC];
  if (tid == 0) s_bad = 0;
  // smallest and largest |pivot|^2 of the steps this thread selects (the
  // threads with ti == 0 select the pivots of their column group)
  double pmin = INFINITY, pmax = 0.0;
  double2 a[RR][RC];
  bool un[RR];   // this thread's rows not pivoted yet
#pragma unroll
  for (int ra = 0; ra < RR; ++ra) {
    const int i = ti + TR * ra;
    un[ra] = i < p;
#pragma unroll
    for (int ca = 0; ca < RC; ++ca) {
      const int j = tj + TC * ca;
      const int64_t o = (sym && j > i) ? (int64_t)j * n + i : (int64_t)i * n + j;
      a[ra][ca] = (i < p && j < p) ? ld2(F.core + o) : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // ---- phase A: LU with implicit row pivoting
#pragma unroll
  for (int kq = 0; kq < RC; ++kq) {
    for (int kc = 0; kc < TC; ++kc) {
      const int k = kq * TC + kc;
      if (k >= p) break;
      if (tj == kc) {
        // largest unused row of column k (ties: lowest row); row k itself in
        // symmetric mode.  bi == p means "no unused row seen"; any unused row
        // replaces it, so the search returns an unused row even when the
        // column holds NaNs (which no comparison selects); a NaN or zero
        // pivot is then flagged.
        double bv = -1.0;
        int bi = p;
#pragma unroll
        for (int ra = 0; ra < RR; ++ra) {
          const double2 v = a[ra][kq];
          const double m = v.x * v.x + v.y * v.y;
          const int i = ti + TR * ra;
          if (un[ra] && (sym ? i == k : (bi == p || m > bv))) { bv = m; bi = i; }
        }
#pragma unroll
        for (int off = TR / 2; off > 0; off >>= 1) {
          const double ov = __shfl_xor(bv, off, TR);
          const int oi = __shfl_xor(bi, off, TR);
          if (oi != p && (bi == p || ov > bv || (ov == bv && oi < bi))) { bv = ov; bi = oi; }
        }
        if (ti == 0) {
          if (!(bv > 0.0) || !(bv < INFINITY)) s_bad = 1;
          pmin = fmin(pmin, bv);
          pmax = fmax(pmax, bv);
          s_r = bi;
          piv_row[k] = bi;
          piv_step[bi] = k;
        }
      }
      __syncthreads();
      // the pivot column and row go through LDS between the two barriers (the
      // previous step's reads of both buffers finished before the first)
      const int r = s_r, rr = r % TR, rq = r / TR;
      if (tj == kc) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra) {
          const int i = ti + TR * ra;
          if (i < p) colbuf[i] = a[ra][kq];
        }
      }
      if (ti == rr) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra)
          if (ra == rq) {
#pragma unroll
            for (int ca = 0; ca < RC; ++ca) {
              const int j = tj + TC * ca;
              if (j < p) rowbuf[j] = a[ra][ca];
            }
          }
      }
#pragma unroll
      for (int ra = 0; ra < RR; ++ra) un[ra] = un[ra] && (ti + TR * ra != r);
      __syncthreads();
      const double2 inv = cinv(rowbuf[k]);
      double2 l[RR], u[RC];
#pragma unroll
      for (int ra = 0; ra < RR; ++ra) l[ra] = un[ra] ? cmul(colbuf[ti + TR * ra], inv) : make_double2(0.0, 0.0);
      // register columns ca < kq hold only j < k: nothing to update there
#pragma unroll
      for (int ca = kq; ca < RC; ++ca) {
        const int j = tj + TC * ca;
        u[ca] = (j > k && j < p) ? rowbuf[j] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int ra = 0; ra < RR; ++ra)
#pragma unroll
        for (int ca = kq; ca < RC; ++ca) {
          double2 v = a[ra][ca];
          v.x = fma(-l[ra].x, u[ca].x, fma(l[ra].y, u[ca].y, v.x));
          v.y = fma(-l[ra].x, u[ca].y, fma(-l[ra].y, u[ca].x, v.y));
          a[ra][ca] = v;
        }
      if (tj == kc) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra)
          if (un[ra]) a[ra][kq] = l[ra];
      }
    }
  }
  if (ti == 0) {
    s_pmin[tj] = pmin;
    s_pmax[tj] = pmax;
  }
  __syncthreads();
  // pivot spread of the block, min |u_kk| / max |u_kk| (a near-singular block
  // shows as a small value)
  if (tid == 0 && pivq) {
    double lo = INFINITY, hi = 0.0;
    for (int c = 0; c < TC; ++c) {
      lo = fmin(lo, s_pmin[c]);
      hi = fmax(hi, s_pmax[c]);
    }
    pivq[ids[blockIdx.x]] = (hi > 0.0 && lo <= hi) ? sqrt(lo / hi) : 0.0;
  }
  // ---- phase B: in-place inverses of L and U, in step order
  int st[RR];
#pragma unroll
  for (int ra = 0; ra < RR; ++ra) {
    const int i = ti + TR * ra;
    st[ra] = i < p ? piv_step[i] : INV_MAXP;
  }
#pragma unroll
  for (int kq = 0; kq < RC; ++kq) {
    for (int kc = 0; kc < TC; ++kc) {
      const int k = kq * TC + kc;
      if (k >= p) break;
      const int r = piv_row[k], rr = r % TR, rq = r / TR;
      if (ti == rr) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra)
          if (ra == rq) {
#pragma unroll
            for (int ca = 0; ca < RC; ++ca) {
              const int j = tj + TC * ca;
              if (j < p) rowbuf[j] = a[ra][ca];
            }
          }
      }
      if (tj == kc) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra) {
          const int i = ti + TR * ra;
          if (i < p) colbuf[i] = a[ra][kq];
        }
      }
      __syncthreads();
      const double2 inv = cinv(rowbuf[k]);
      // entry (i, j) takes c_i * s_j when i > k > j (L triangle, s_j = row_k[j])
      // or i < k < j (U triangle, s_j = row_k[j] / u_kk): the row side and
      // the column side must agree
      // register columns ca < kq hold j < k (L side), ca > kq hold j > k (U
      // side); column kq holds j = tj + TC kq, on either side of k.  mL / mU:
      // the column factor c_i of rows that take the L / U update (zero else);
      // entries j >= p have s_j = 0.
      double2 mL[RR], mU[RR], sv[RC];
#pragma unroll
      for (int ra = 0; ra < RR; ++ra) {
        const int i = ti + TR * ra;
        const double2 c = i < p ? colbuf[i] : make_double2(0.0, 0.0);
        const bool lrow = st[ra] > k && st[ra] < INV_MAXP, urow = st[ra] < k;
        mL[ra] = lrow ? c : make_double2(0.0, 0.0);
        mU[ra] = urow ? c : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int ca = 0; ca < RC; ++ca) {
        const int j = tj + TC * ca;
        const double2 rj = j < p ? rowbuf[j] : make_double2(0.0, 0.0);
        sv[ca] = j < k ? rj : cmul(rj, inv);
      }
#pragma unroll
      for (int ra = 0; ra < RR; ++ra)
#pragma unroll
        for (int ca = 0; ca < RC; ++ca) {
          double2 m;
          if (ca < kq) m = mL[ra];
          else if (ca > kq) m = mU[ra];
          else m = tj < kc ? mL[ra] : (tj > kc ? mU[ra] : make_double2(0.0, 0.0));
          double2 v = a[ra][ca];
          v.x = fma(-m.x, sv[ca].x, fma(m.y, sv[ca].y, v.x));
          v.y = fma(-m.x, sv[ca].y, fma(-m.y, sv[ca].x, v.y));
          a[ra][ca] = v;
        }
      // row k: scale its U part; column k: negate (L) or negate and scale (U)
      if (ti == rr) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra)
          if (ra == rq) {
#pragma unroll
            for (int ca = 0; ca < RC; ++ca) {
              const int j = tj + TC * ca;
              if (j > k && j < p) a[ra][ca] = sv[ca];
            }
          }
      }
      if (tj == kc) {
#pragma unroll
        for (int ra = 0; ra < RR; ++ra) {
          const int i = ti + TR * ra;
          if (i < p) {
            const double2 c = colbuf[i];
            if (st[ra] > k) a[ra][kq] = make_double2(-c.x, -c.y);
            else if (st[ra] < k) a[ra][kq] = make_double2(-(c.x * inv.x - c.y * inv.y), -(c.x * inv.y + c.y * inv.x));
            else a[ra][kq] = inv;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0 && s_bad) atomicOr(status, ST_SINGULAR);
  for (int k = tid; k < p; k += TR * TC) F.perm[k] = piv_row[k];
#pragma unroll
  for (int ra = 0; ra < RR; ++ra)
#pragma unroll
    for (int ca = 0; ca < RC; ++ca) {
      const int x = ti + TR * ra, y = tj + TC * ca;
      if (x < p && y < p) st2(F.tri + (int64_t)st[ra] * p + y, a[ra][ca]);
    }
}

// ---------------------------------------------------------------------------
// Batched complex FP64 GEMM on MFMA: one 64x64 output tile per workgroup of
// four waves; each wave owns a 32x32 quadrant as 2x2 blocks of 16x16, with
// the real and imaginary parts in separate accumulators (four real
// v_mfma_f64_16x16x4 per complex block and k-step of 4).
// ---------------------------------------------------------------------------
constexpr int KT = 16;

// Entry of a packed triangular operand at stored position (r, c): the strict
// lower part with a unit diagonal (lower) or the upper part with its diagonal.
__device__ __forceinline__ double2 tri_mask(bool lower, int r, int c, bool inside, double2 v) {
  if (!inside) return make_double2(0.0, 0.0);
  if (lower) return r > c ? v : (r == c ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0));
  return r <= c ? v : make_double2(0.0, 0.0);
}

// MFMA flavours of the GEMM: FP64 (v_mfma_f64_16x16x4) or FP32 with FP32
// accumulation (v_mfma_f32_16x16x4) on operands rounded to FP32 when they are
// staged in LDS; memory operands and results stay FP64 either way.
template <bool F32>
struct GemmPrec;
template <>
struct GemmPrec<false> {
  typedef double2 lds_t;
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // D layout: lane l, element q -> row (l/16) + 4q, column l%16
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
  static __device__ __forceinline__ lds_t cvt(double2 v) { return v; }
  // LDS column swizzle of A (16-byte entries, 8 per 128-byte bank row)
  static __device__ __forceinline__ int swz(int k) { return ((k >> 2) & 3) << 1; }
};
template <>
struct GemmPrec<true> {
  typedef float2 lds_t;
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // D layout: lane l, element q -> row 4(l/16) + q, column l%16
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
  static __device__ __forceinline__ lds_t cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
  // LDS column swizzle of A (8-byte entries, 16 per 128-byte bank row)
  static __device__ __forceinline__ int swz(int k) { return ((k >> 2) & 3) << 2; }
};

// One 64x64 output tile.  TRI: the task has a triangular operand (masked
// loads, zero blocks of the triangle skipped); the other instantiation has
// none of that code.  K3 (FP64 only): complex products from three real
// products instead of four (Karatsuba): with a = ar + i ai, b = br + i bi,
//   k1 = (ar + ai) br,  k2 = ar (bi - br),  k3 = ai (br + bi),
//   re(ab) = k1 - k3,   im(ab) = k1 + k2,
// each k summed over K in its own accumulator; a quarter fewer MFMAs for
// a third more accumulator registers.
template <bool F32, bool TRI, bool K3 = false>
__device__ __forceinline__ void gemm_tile(const GemmTask &T, int coff, int N, int nlimk, const cplx *ext,
                                          double *part, int pstride, typename GemmPrec<F32>::lds_t (*As)[64],
                                          typename GemmPrec<F32>::lds_t (*Bs)[64]) {
  typedef GemmPrec<F32> GP;
  typedef typename GP::lds_t lds_t;
  typedef typename GP::acc_t acc_t;
  const int M = T.M, K = ((T.flags & G_K_LIM) && nlimk < T.K) ? nlimk : T.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool transA = T.flags & G_TRANS_A;
  const cplx *Bp = (T.flags & G_B_EXT) ? ext + reinterpret_cast<intptr_t>(T.B) : T.B;
  if (T.flags & G_B_COFF) Bp += coff;
  cplx *Cp = (T.flags & G_C_EXT) ? const_cast<cplx *>(ext) : T.C;
  if (T.flags & G_C_COFF) Cp += coff;

  static_assert(!(K3 && F32), "the three-product form is for the FP64 path");
  // four-product form: cre, cim; three-product form: k1 -> cre, k2 -> cim, k3
  acc_t cre[2][2], cim[2][2], ck3[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      cre[r][c] = acc_t{0, 0, 0, 0};
      cim[r][c] = acc_t{0, 0, 0, 0};
      ck3[r][c] = acc_t{0, 0, 0, 0};
    }
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  // k range that can hold nonzeros when an operand is triangular
  const int fl = T.flags;
  int kbeg = 0, kend = K;
  if (fl & G_A_TRI_L) { if (transA) kbeg = T.tm; else kend = min(kend, T.tm + 64); }
  if (fl & G_A_TRI_U) { if (transA) kend = min(kend, T.tm + 64); else kbeg = T.tm; }
  if (fl & G_B_TRI_L) kbeg = max(kbeg, T.tn);
  if (fl & G_B_TRI_U) kend = min(kend, T.tn + 64);
  kbeg = (kbeg / KT) * KT;
  const bool triA = TRI && (fl & (G_A_TRI_L | G_A_TRI_U)), triB = TRI && (fl & (G_B_TRI_L | G_B_TRI_U));
  // nonzero pattern of a triangular operand in (i, k) / (k, j) terms:
  // 1 = nonzero only for k <= i (k <= j), 2 = only for k >= i (k >= j)
  const int akind = !triA ? 0 : ((((fl & G_A_TRI_L) != 0) != transA) ? 1 : 2);
  const int bkind = !triB ? 0 : ((fl & G_B_TRI_L) ? 2 : 1);

  // interior tiles (no edge in M or N) load a k slab without per-element
  // conditions when the slab is full in K and, for a triangular operand,
  // lies strictly on the nonzero side of its diagonal (raw stored values)
  const bool interior = T.tm + 64 <= M && T.tn + 64 <= N;
  auto slab_raw = [&](int k0) -> bool {
    if (!interior || k0 + KT > K) return false;
    if (triA && !(akind == 1 ? k0 + KT - 1 < T.tm : k0 > T.tm + 63)) return false;
    if (triB && !(bkind == 1 ? k0 + KT - 1 < T.tn : k0 > T.tn + 63)) return false;
    return true;
  };
  // 16x16 output blocks of this wave that hold any output entry
  bool blk_ok[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) blk_ok[r][c] = T.tm + wr + 16 * r < M && T.tn + wc + 16 * c < N;
  // FP64 tiles without a triangular operand: k stages of 8 loaded straight
  // into LDS (no register staging), two stages in flight, one barrier per
  // stage.  At a tile's edge the rows and columns past M and N load copies
  // of the last row and column (their results are computed and not stored),
  // so that the MFMA loop is the interior tiles' own.  Stage 0 lives in As,
  // stage 1 in Bs (two distinct LDS objects, so that the compiler sees the
  // MFMA operand reads of one stage as independent of the loads in flight
  // into the other): entries [0, 512) hold the A slab, [512, 1024) the B
  // slab.  B and a
  // transposed-stored A are [k][64] rows; a row-major A is [i][8] with entry
  // (i, k) at i*8 + (k ^ ((i >> 1) & 7)), so that both the coalesced loads (8
  // lanes per row) and the MFMA operand reads (16 rows at one k) meet every
  // LDS bank once.
  constexpr int KD = 8;
  bool dma = false;
  if constexpr (!F32 && !TRI) {
    if (K >= 2 * KD) {
      dma = true;
      double2 *S0 = &As[0][0], *S1 = &Bs[0][0];
      const int nfull = K / KD, tail = K - nfull * KD;
      // the wave index as a scalar, and the row map read through the constant
      // address space: the B row indices of a stage are then scalar loads,
      // which do not wait for the stage loads in flight
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      typedef __attribute__((address_space(4))) const int32_t cint;
      cint *bmap = (cint *)T.browmap;
      // B column and transposed-A column of this lane, row-major A rows of
      // its two blocks, clamped to the operands' last column / row
      const int bj = min(T.tn + lane, N - 1), at = min(T.tm + lane, M - 1);
      int ar[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) ar[q] = min(T.tm + 8 * (2 * wv + q) + (lane >> 3), M - 1);
      int ao[2][2], bo[2][2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int kx = 4 * ks + (lane >> 4), i = wr + 16 * r + (lane & 15);
          ao[ks][r] = transA ? kx * 64 + i : i * 8 + (kx ^ ((i >> 1) & 7));
          bo[ks][r] = 512 + kx * 64 + wc + 16 * r + (lane & 15);
        }
      auto issue = [&](int k0, double2 *buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int kr = 2 * wv + q, gk = k0 + kr;
          ld_lds16(Bp + (int64_t)(bmap ? bmap[gk] : gk) * T.ldb + bj, buf + 512 + kr * 64);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int blk = 2 * wv + q;
          if (transA) {
            ld_lds16(T.A + (int64_t)(k0 + blk) * T.lda + at, buf + blk * 64);
          } else {
            const int i = 8 * blk + (lane >> 3), k = (lane & 7) ^ ((i >> 1) & 7);
            ld_lds16(T.A + (int64_t)ar[q] * T.lda + k0 + k, buf + blk * 64);
          }
        }
      };
      // the last, partial stage: plain loads, zeros past K, M and N
      auto fill_tail = [&](int k0, double2 *buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int e = tid + 256 * q;
          {
            const int kr = e >> 6, j = e & 63, gk = k0 + kr;
            buf[512 + kr * 64 + j] = (gk < K && T.tn + j < N)
                                         ? ld2(Bp + (int64_t)(T.browmap ? T.browmap[gk] : gk) * T.ldb + T.tn + j)
                                         : make_double2(0.0, 0.0);
          }
          if (transA) {
            const int kr = e >> 6, i = e & 63, gk = k0 + kr;
            buf[kr * 64 + i] = (gk < K && T.tm + i < M) ? ld2(T.A + (int64_t)gk * T.lda + T.tm + i)
                                                        : make_double2(0.0, 0.0);
          } else {
            const int i = e >> 3, k = e & 7, gk = k0 + k;
            buf[i * 8 + (k ^ ((i >> 1) & 7))] = (gk < K && T.tm + i < M) ? ld2(T.A + (int64_t)(T.tm + i) * T.lda + gk)
                                                                         : make_double2(0.0, 0.0);
          }
        }
      };
      auto compute = [&](const double2 *buf) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          double2 a[2], b[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            a[r] = buf[ao[ks][r]];
            b[r] = buf[bo[ks][r]];
          }
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              if constexpr (K3) {
                cre[r][c] = GP::mfma(a[r].x + a[r].y, b[c].x, cre[r][c]);
                cim[r][c] = GP::mfma(a[r].x, b[c].y - b[c].x, cim[r][c]);
                ck3[r][c] = GP::mfma(a[r].y, b[c].x + b[c].y, ck3[r][c]);
              } else {
                cre[r][c] = GP::mfma(a[r].x, b[c].x, cre[r][c]);
                cre[r][c] = GP::mfma(-a[r].y, b[c].y, cre[r][c]);
                cim[r][c] = GP::mfma(a[r].x, b[c].y, cim[r][c]);
                cim[r][c] = GP::mfma(a[r].y, b[c].x, cim[r][c]);
              }
            }
        }
      };
      // stage s in S0 (s even) or S1 (s odd): this wave's loads of stage s,
      // then every wave's (and every wave done with the buffer the next
      // stage overwrites), then the next stage's loads, then the MFMAs
      issue(0, S0);
      for (int s = 0; s < nfull; s += 2) {
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        if (s + 1 < nfull)
          issue((s + 1) * KD, S1);
        else if (tail)
          fill_tail(nfull * KD, S1);
        compute(S0);
        if (s + 1 < nfull) {
          __builtin_amdgcn_s_waitcnt(0x0F70);
          __syncthreads();
          if (s + 2 < nfull)
            issue((s + 2) * KD, S0);
          else if (tail)
            fill_tail(nfull * KD, S0);
          compute(S1);
        }
      }
      if (tail) {
        __syncthreads();
        compute((nfull & 1) ? S1 : S0);
      }
    }
  }
  for (int k0 = dma ? kend : kbeg; k0 < kend; k0 += KT) {
    double2 ra[4], rb[4];
    if (slab_raw(k0)) {
      if (!transA) {
        const int i = tid >> 2, kq = (tid & 3) * 4;
        const gcplx *a = as_global(T.A) + (int64_t)(T.tm + i) * T.lda + k0 + kq;
        for (int q = 0; q < 4; ++q) ra[q] = ldg(a + q);
      } else {
        const int k = tid >> 4, i0 = tid & 15;
        const gcplx *a = as_global(T.A) + (int64_t)(k0 + k) * T.lda + T.tm + i0;
        for (int q = 0; q < 4; ++q) ra[q] = ldg(a + 16 * q);
      }
      {
        const int k = tid >> 4, j0 = tid & 15;
        const int gk = k0 + k;
        const gcplx *b = as_global(Bp) + (int64_t)(T.browmap ? T.browmap[gk] : gk) * T.ldb + T.tn + j0;
        for (int q = 0; q < 4; ++q) rb[q] = ldg(b + 16 * q);
      }
    } else {
      if (!transA) {
        const int i = tid >> 2, kq = (tid & 3) * 4;
        const int gi = T.tm + i;
        for (int q = 0; q < 4; ++q) {
          const int gk = k0 + kq + q;
          ra[q] = (gi < M && gk < K) ? ld2(T.A + (int64_t)gi * T.lda + gk) : make_double2(0.0, 0.0);
          if (triA) ra[q] = tri_mask(fl & G_A_TRI_L, gi, gk, gi < M && gk < K, ra[q]);
        }
      } else {
        // stored k-major: 16 lanes read 16 consecutive entries of one row
        const int k = tid >> 4, i0 = tid & 15;
        const int gk = k0 + k;
        for (int q = 0; q < 4; ++q) {
          const int gi = T.tm + i0 + 16 * q;
          ra[q] = (gi < M && gk < K) ? ld2(T.A + (int64_t)gk * T.lda + gi) : make_double2(0.0, 0.0);
          if (triA) ra[q] = tri_mask(fl & G_A_TRI_L, gk, gi, gi < M && gk < K, ra[q]);
        }
      }
      {
        const int k = tid >> 4, j0 = tid & 15;
        const int gk = k0 + k;
        const cplx *row = nullptr;
        if (gk < K) row = Bp + (int64_t)(T.browmap ? T.browmap[gk] : gk) * T.ldb;
        for (int q = 0; q < 4; ++q) {
          const int gj = T.tn + j0 + 16 * q;
          rb[q] = (row && gj < N) ? ld2(row + gj) : make_double2(0.0, 0.0);
          if (triB) rb[q] = tri_mask(fl & G_B_TRI_L, gk, gj, gk < K && gj < N, rb[q]);
        }
      }
    }
    __syncthreads();
    // As columns are XOR-swizzled by GP::swz(k): the transposing stores of a
    // row-major A then spread over all LDS banks, and a row read stays
    // conflict-free (the swizzle permutes within aligned groups of columns)
    if (!transA) {
      const int i = tid >> 2, kq = (tid & 3) * 4;
      for (int q = 0; q < 4; ++q) As[kq + q][i ^ GP::swz(kq + q)] = GP::cvt(ra[q]);
    } else {
      const int k = tid >> 4, i0 = tid & 15;
      for (int q = 0; q < 4; ++q) As[k][(i0 + 16 * q) ^ GP::swz(k)] = GP::cvt(ra[q]);
    }
    {
      const int k = tid >> 4, j0 = tid & 15;
      for (int q = 0; q < 4; ++q) Bs[k][j0 + 16 * q] = GP::cvt(rb[q]);
    }
    __syncthreads();
    // 16x16 blocks that take part in this slab: inside the output and, for a
    // triangular operand, not zero over the whole slab (wave-uniform)
    bool ok[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        ok[r][c] = blk_ok[r][c];
        if (TRI) {
          const int i0 = T.tm + wr + 16 * r, j0 = T.tn + wc + 16 * c, k1 = k0 + KT - 1;
          if (akind == 1 && k0 > i0 + 15) ok[r][c] = false;
          if (akind == 2 && k1 < i0) ok[r][c] = false;
          if (bkind == 1 && k0 > j0 + 15) ok[r][c] = false;
          if (bkind == 2 && k1 < j0) ok[r][c] = false;
        }
      }
    const bool ok_all = ok[0][0] && ok[0][1] && ok[1][0] && ok[1][1];
    if (ok_all && k0 + KT <= kend) {
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const int kx = kk + (lane >> 4);
        lds_t a[2], b[2];
        a[0] = As[kx][(wr + (lane & 15)) ^ GP::swz(kx)];
        a[1] = As[kx][(wr + 16 + (lane & 15)) ^ GP::swz(kx)];
        b[0] = Bs[kx][wc + (lane & 15)];
        b[1] = Bs[kx][wc + 16 + (lane & 15)];
        if constexpr (K3) {
          double as[2], bd[2], bs[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) as[r] = a[r].x + a[r].y;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            bd[c] = b[c].y - b[c].x;
            bs[c] = b[c].x + b[c].y;
          }
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              cre[r][c] = GP::mfma(as[r], b[c].x, cre[r][c]);
              cim[r][c] = GP::mfma(a[r].x, bd[c], cim[r][c]);
              ck3[r][c] = GP::mfma(a[r].y, bs[c], ck3[r][c]);
            }
        } else {
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              cre[r][c] = GP::mfma(a[r].x, b[c].x, cre[r][c]);
              cre[r][c] = GP::mfma(-a[r].y, b[c].y, cre[r][c]);
              cim[r][c] = GP::mfma(a[r].x, b[c].y, cim[r][c]);
              cim[r][c] = GP::mfma(a[r].y, b[c].x, cim[r][c]);
            }
        }
      }
    } else {
      // edge tile, zero triangle blocks or last slab: skip the blocks that do
      // not take part and the k steps past the end of the k range
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        if (k0 + kk >= kend) break;
        const int kx = kk + (lane >> 4);
        lds_t a[2], b[2];
        a[0] = As[kx][(wr + (lane & 15)) ^ GP::swz(kx)];
        a[1] = As[kx][(wr + 16 + (lane & 15)) ^ GP::swz(kx)];
        b[0] = Bs[kx][wc + (lane & 15)];
        b[1] = Bs[kx][wc + 16 + (lane & 15)];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (ok[r][c]) {
              if constexpr (K3) {
                cre[r][c] = GP::mfma(a[r].x + a[r].y, b[c].x, cre[r][c]);
                cim[r][c] = GP::mfma(a[r].x, b[c].y - b[c].x, cim[r][c]);
                ck3[r][c] = GP::mfma(a[r].y, b[c].x + b[c].y, ck3[r][c]);
              } else {
                cre[r][c] = GP::mfma(a[r].x, b[c].x, cre[r][c]);
                cre[r][c] = GP::mfma(-a[r].y, b[c].y, cre[r][c]);
                cim[r][c] = GP::mfma(a[r].x, b[c].y, cim[r][c]);
                cim[r][c] = GP::mfma(a[r].y, b[c].x, cim[r][c]);
              }
            }
      }
    }
  }

  const bool neg = T.flags & G_NEG;
  const bool store = !(T.flags & G_NO_STORE), contract = T.flags & G_CONTRACT;
  const cplx *Cin = (T.flags & G_CIN) ? T.Cin : nullptr;
  if (Cin && (T.flags & G_CIN_COFF)) Cin += coff;
  // G_CIN_RANGE: Cin column of output column j, or -1 where Cin is zero
  const bool crange = T.flags & G_CIN_RANGE;
  const int cshift = coff - T.cin_c0;
  // Epilogue in three passes (results, stores, contraction), so that the
  // loads of each pass are all in flight together.  Lane l holds rows
  // row(l, q) of the 16-row blocks r and columns l % 16 of the blocks c.
  const bool own = T.flags & G_CIN_OWN;
  int64_t oi[2][4], ci[2][4];
  bool rowok[2][4], addold[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gi = T.tm + wr + 16 * r + GP::row(lane, q);
      rowok[r][q] = gi < M;
      const int32_t m = (rowok[r][q] && T.crowmap) ? T.crowmap[gi] : gi;
      oi[r][q] = rowok[r][q] ? (m & EXT_ROW_MASK) : 0;
      addold[r][q] = (m & EXT_ADD) != 0;
      ci[r][q] = own ? gi : oi[r][q];
    }
  bool colok[2];
  int oj[2];   // output column (mapped through ccolmap)
  const bool cacc = (T.flags & G_C_ACC) || ((T.flags & G_ACC_CHUNK) && coff > 0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int gj = T.tn + wc + 16 * c + (lane & 15);
    colok[c] = gj < N;
    oj[c] = (colok[c] && T.ccolmap) ? T.ccolmap[gj] : gj;
  }
  double2 v[2][2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gj = T.tn + wc + 16 * c + (lane & 15);
        if constexpr (K3)
          v[r][c][q] = make_double2(cre[r][c][q] - ck3[r][c][q], cre[r][c][q] + cim[r][c][q]);
        else
          v[r][c][q] = make_double2((double)cre[r][c][q], (double)cim[r][c][q]);
        if (neg) v[r][c][q] = make_double2(-v[r][c][q].x, -v[r][c][q].y);
        if (crange) {
          const int cj = gj + cshift;
          if (Cin && rowok[r][q] && colok[c] && cj >= 0 && cj < T.cin_w)
            v[r][c][q] = cadd(v[r][c][q], ld2(Cin + ci[r][q] * T.ldcin + cj));
        } else if (Cin && rowok[r][q] && colok[c]) {
          v[r][c][q] = cadd(v[r][c][q], ld2(Cin + ci[r][q] * T.ldcin + (own ? gj : oj[c])));
        }
        if ((addold[r][q] || cacc) && rowok[r][q] && colok[c])
          v[r][c][q] = cadd(v[r][c][q], ld2(Cp + oi[r][q] * T.ldc + oj[c]));
      }
  if (store) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rowok[r][q] && colok[c]) st2(Cp + oi[r][q] * T.ldc + oj[c], v[r][c][q]);
  }
  if (contract) {
    // gradient partials: per row, Re(C aux) summed over the wave's 32 columns
    double acc[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[r][q] = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
          if (rowok[r][q] && colok[c]) {
            const double2 y = ld2(T.aux + oi[r][q] * T.ldc + T.tn + wc + 16 * c + (lane & 15));
            acc[r][q] += v[r][c][q].x * y.x - v[r][c][q].y * y.y;
          }
      }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double a = acc[r][q];
        for (int off = 1; off < 16; off <<= 1) a += __shfl_xor(a, off, 64);
        if ((lane & 15) == 0 && rowok[r][q]) {
          const int g = T.auxmap[oi[r][q]];
          if (g >= 0) part[(int64_t)((coff + T.tn + wc) / 32) * pstride + g] = a;
        }
      }
  }
}

// FP64 tiles whose valid rows fit in RB (1 or 2) blocks of 16: the small
// separator fronts near the leaves (p of 8 to 32 pivots), the leaves' L21 and
// Z products (b up to 32 rows, a triangular operand) and ragged last row
// tiles.  In the 2x2 wave layout of gemm_tile such a tile leaves half of its
// waves without a block and stages every k slab through LDS behind two
// barriers, so its time is a chain of load round trips.  Here wave w owns the
// 16 columns [16w, 16w + 16) of the tile and all RB row blocks, and loads its
// MFMA operands from global memory straight into registers, KS k-steps of 4
// at a time, with no LDS and no barrier in the k loop (A, a few KB per front,
// is read by every wave, from cache).  Same task semantics and epilogue as
// gemm_tile; the contraction's 32-column partials combine the row sums of
// waves 2g and 2g + 1 through LDS (red: 4 x 16 RB doubles).
template <int RB, int KS, bool TRI, bool F32>
__device__ __forceinline__ void thin_tile(const GemmTask &T, int coff, int N, int nlimk, const cplx *ext,
                                          double *part, int pstride, double *red) {
  typedef GemmPrec<F32> GP;
  typedef typename GP::acc_t acc_t;
  const int M = T.M, K = ((T.flags & G_K_LIM) && nlimk < T.K) ? nlimk : T.K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const bool transA = T.flags & G_TRANS_A;
  const cplx *Bp = (T.flags & G_B_EXT) ? ext + reinterpret_cast<intptr_t>(T.B) : T.B;
  if (T.flags & G_B_COFF) Bp += coff;
  cplx *Cp = (T.flags & G_C_EXT) ? const_cast<cplx *>(ext) : T.C;
  if (T.flags & G_C_COFF) Cp += coff;
  const int wc = 16 * wave;
  // MFMA operands of lane l: A(row l % 16 of a block, k = l / 16 of a step),
  // B(k = l / 16, column l % 16)
  const int bj = T.tn + wc + li;
  const bool bjok = bj < N;
  int ai[RB];
  bool aiok[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    ai[r] = T.tm + 16 * r + li;
    aiok[r] = ai[r] < M;
  }
  acc_t cre[RB], cim[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    cre[r] = acc_t{0, 0, 0, 0};
    cim[r] = acc_t{0, 0, 0, 0};
  }
  // a triangular operand: masked loads (the stored-triangle rules of
  // tri_mask) and the k range that can hold nonzeros for this tile's rows and
  // this wave's columns, from a k-step boundary
  const int fl = T.flags;
  const bool triA = TRI && (fl & (G_A_TRI_L | G_A_TRI_U)), triB = TRI && (fl & (G_B_TRI_L | G_B_TRI_U));
  int kbeg = 0, kend = K;
  if (TRI) {
    if (fl & G_A_TRI_L) { if (transA) kbeg = T.tm; else kend = min(kend, T.tm + 16 * RB); }
    if (fl & G_A_TRI_U) { if (transA) kend = min(kend, T.tm + 16 * RB); else kbeg = T.tm; }
    if (fl & G_B_TRI_L) kbeg = max(kbeg, T.tn + wc);
    if (fl & G_B_TRI_U) kend = min(kend, T.tn + wc + 16);
    kbeg &= ~3;
  }
  const bool wave_cols = T.tn + wc < N;   // the wave holds any output column
  if (wave_cols) {
    for (int k0 = kbeg; k0 < kend; k0 += 4 * KS) {
      double2 a[KS][RB], b[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int gk = k0 + 4 * s + lk;
        const bool kok = gk < kend;
        const int br = kok ? (T.browmap ? T.browmap[gk] : gk) : 0;
        b[s] = (kok && bjok) ? ldg(as_global(Bp) + (int64_t)br * T.ldb + bj) : make_double2(0.0, 0.0);
        if (triB) b[s] = tri_mask(fl & G_B_TRI_L, gk, bj, kok && bjok, b[s]);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          a[s][r] = (kok && aiok[r])
                        ? ldg(as_global(T.A) + (transA ? (int64_t)gk * T.lda + ai[r] : (int64_t)ai[r] * T.lda + gk))
                        : make_double2(0.0, 0.0);
          if (triA)
            a[s][r] = transA ? tri_mask(fl & G_A_TRI_L, gk, ai[r], kok && aiok[r], a[s][r])
                             : tri_mask(fl & G_A_TRI_L, ai[r], gk, kok && aiok[r], a[s][r]);
        }
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        if (k0 + 4 * s >= kend) break;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          // (FP32: operands rounded as the LDS stages of gemm_tile round them)
          const auto av = GP::cvt(a[s][r]), bv = GP::cvt(b[s]);
          cre[r] = GP::mfma(av.x, bv.x, cre[r]);
          cre[r] = GP::mfma(-av.y, bv.y, cre[r]);
          cim[r] = GP::mfma(av.x, bv.y, cim[r]);
          cim[r] = GP::mfma(av.y, bv.x, cim[r]);
        }
      }
    }
  }

  // epilogue: lane l holds rows (l / 16) + 4q of each row block, column l % 16
  const bool neg = T.flags & G_NEG;
  const bool store = !(T.flags & G_NO_STORE), contract = T.flags & G_CONTRACT;
  const cplx *Cin = (T.flags & G_CIN) ? T.Cin : nullptr;
  if (Cin && (T.flags & G_CIN_COFF)) Cin += coff;
  const bool crange = T.flags & G_CIN_RANGE;
  const int cshift = coff - T.cin_c0;
  const bool own = T.flags & G_CIN_OWN;
  const bool cacc = (T.flags & G_C_ACC) || ((T.flags & G_ACC_CHUNK) && coff > 0);
  const int gj = bj;
  const bool colok = bjok;
  const int oj = (colok && T.ccolmap) ? T.ccolmap[gj] : gj;
  double2 v[RB][4];
  int64_t oi[RB][4];
  bool rowok[RB][4];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gi = T.tm + 16 * r + GP::row(lane, q);
      rowok[r][q] = gi < M;
      const int32_t m = (rowok[r][q] && T.crowmap) ? T.crowmap[gi] : gi;
      oi[r][q] = rowok[r][q] ? (m & EXT_ROW_MASK) : 0;
      const bool addold = (m & EXT_ADD) != 0;
      const int64_t ci = own ? gi : oi[r][q];
      double2 x = make_double2((double)cre[r][q], (double)cim[r][q]);
      if (neg) x = make_double2(-x.x, -x.y);
      if (crange) {
        const int cj = gj + cshift;
        if (Cin && rowok[r][q] && colok && cj >= 0 && cj < T.cin_w) x = cadd(x, ld2(Cin + ci * T.ldcin + cj));
      } else if (Cin && rowok[r][q] && colok) {
        x = cadd(x, ld2(Cin + ci * T.ldcin + (own ? gj : oj)));
      }
      if ((addold || cacc) && rowok[r][q] && colok) x = cadd(x, ld2(Cp + oi[r][q] * T.ldc + oj));
      v[r][q] = x;
    }
  if (store) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (rowok[r][q] && colok) st2(Cp + oi[r][q] * T.ldc + oj, v[r][q]);
  }
  if (contract) {
    // row sums of Re(C aux) over the wave's 16 columns, then over the pair of
    // waves that shares a 32-column partial
    double acc[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double a = 0.0;
        if (rowok[r][q] && colok) {
          const double2 y = ld2(T.aux + oi[r][q] * T.ldc + gj);
          a = v[r][q].x * y.x - v[r][q].y * y.y;
        }
        for (int off = 1; off < 16; off <<= 1) a += __shfl_xor(a, off, 64);
        acc[r][q] = a;
      }
    if ((wave & 1) && li == 0) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(wave >> 1) * 16 * RB + 16 * r + GP::row(lane, q)] = acc[r][q];
    }
    __syncthreads();
    if (!(wave & 1) && li == 0) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rowok[r][q]) {
            const int g = T.auxmap[oi[r][q]];
            if (g >= 0)
              part[(int64_t)((coff + T.tn + 32 * (wave >> 1)) / 32) * pstride + g] =
                  acc[r][q] + red[(wave >> 1) * 16 * RB + 16 * r + GP::row(lane, q)];
          }
    }
  }
}

// The thin tiles of a list (thin_tile_task: at most THIN_ROWS valid rows, no
// triangular operand), which the plan moves to the end of the list, in a
// launch of their own: with neither LDS stages nor the 2x2 layout's
// accumulators this kernel holds twice the workgroups per CU of k_gemm.  A
// thin tile is a short chain of dependent loads (task, row map, operands,
// epilogue), so the number of tiles in flight sets its throughput.
template <bool F32>
__global__ __launch_bounds__(256, 8) void k_gemm_thin(const GemmTask *tasks, int coff, int nlim, const cplx *ext,
                                                      double *part, int pstride) {
  __shared__ double red[2 * 16 * 2];
  const GemmTask T = tasks[blockIdx.x];
  const int N = ((T.flags & G_K_LIM) || T.N < nlim) ? T.N : nlim;
  if (T.tn >= N) return;
  if (T.M - T.tm <= 16)
    thin_tile<1, 2, false, F32>(T, coff, N, nlim, ext, part, pstride, red);
  else
    thin_tile<2, 1, false, F32>(T, coff, N, nlim, ext, part, pstride, red);
}

// The thin tiles with a triangular operand (after the others in a list), in
// a kernel of their own so that their masks and k ranges do not cost the
// plain thin tiles registers.
template <bool F32>
__global__ __launch_bounds__(256, 8) void k_gemm_thin_tri(const GemmTask *tasks, int coff, int nlim,
                                                          const cplx *ext, double *part, int pstride) {
  __shared__ double red[2 * 16 * 2];
  const GemmTask T = tasks[blockIdx.x];
  const int N = ((T.flags & G_K_LIM) || T.N < nlim) ? T.N : nlim;
  if (T.tn >= N) return;
  if (T.M - T.tm <= 16)
    thin_tile<1, 2, true, F32>(T, coff, N, nlim, ext, part, pstride, red);
  else
    thin_tile<2, 1, true, F32>(T, coff, N, nlim, ext, part, pstride, red);
}

template <bool F32>
__global__ __launch_bounds__(256, 4) void k_gemm(const GemmTask *tasks, int coff, int nlim, const cplx *ext,
                                                 double *part, int pstride) {
  __shared__ typename GemmPrec<F32>::lds_t As[KT][64];
  __shared__ typename GemmPrec<F32>::lds_t Bs[KT][64];
  const GemmTask T = tasks[blockIdx.x];
  // the launch's column limit applies to N, or to K for G_K_LIM tasks
  const int N = ((T.flags & G_K_LIM) || T.N < nlim) ? T.N : nlim;
  if (T.tn >= N) return;
  if (T.flags & (G_A_TRI_L | G_A_TRI_U | G_B_TRI_L | G_B_TRI_U))
    gemm_tile<F32, true>(T, coff, N, nlim, ext, part, pstride, As, Bs);
  else
    gemm_tile<F32, false>(T, coff, N, nlim, ext, part, pstride, As, Bs);
}

// Launches that hold deep-K tasks (Schur partials, weighted adjoint source,
// the upper levels' fronts and sweeps): MFMA-bound, so the tasks flagged
// G_K3 take the three-product complex form, at three workgroups per CU for
// its accumulators.  Unflagged tasks of such a launch (other problems of a
// merged batch) keep the four-product form, so that every task rounds the
// same way whichever launch runs it.
__global__ __launch_bounds__(256, 3) void k_gemm_k3(const GemmTask *tasks, int coff, int nlim, const cplx *ext,
                                                   double *part, int pstride) {
  __shared__ double2 As[KT][64];
  __shared__ double2 Bs[KT][64];
  const GemmTask T = tasks[blockIdx.x];
  const int N = ((T.flags & G_K_LIM) || T.N < nlim) ? T.N : nlim;
  if (T.tn >= N) return;
  const bool tri = T.flags & (G_A_TRI_L | G_A_TRI_U | G_B_TRI_L | G_B_TRI_U);
  if (T.flags & G_K3) {
    if (tri)
      gemm_tile<false, true, true>(T, coff, N, nlim, ext, part, pstride, As, Bs);
    else
      gemm_tile<false, false, true>(T, coff, N, nlim, ext, part, pstride, As, Bs);
  } else {
    if (tri)
      gemm_tile<false, true, false>(T, coff, N, nlim, ext, part, pstride, As, Bs);
    else
      gemm_tile<false, false, false>(T, coff, N, nlim, ext, part, pstride, As, Bs);
  }
}

// Wt = Y_bnd Lam_bnd^T of the roots of the low-rank sweep subtrees: a b x b
// product (b <= 64) over the right-hand-side columns whose operands are
// gathered rows of the sweep arrays (A rows arowmap, B rows browmap, each
// row k-contiguous).  One workgroup per root, each wave one 32 x 32
// quadrant; every 16-k slab of the 64 A rows and 64 B rows is read from HBM
// once and shared through LDS, and the next slab's loads are issued before
// the current slab's MFMAs so that they are in flight meanwhile.  Rows past
// the front's size are clamped to its last row (their outputs are not
// stored); k past the chunk's width reads zeros.  The chunk's sum is stored,
// or added for column offsets > 0 (later chunks).
__global__ __launch_bounds__(256, 3) void k_lowrank_w(const GemmTask *tasks, int coff, int nlimk) {
  typedef GemmPrec<false> GP;
  __shared__ double2 As[16][64];
  __shared__ double2 Bs[16][64];
  const GemmTask T = tasks[blockIdx.x];
  const int M = T.M, N = T.N, K = nlimk < T.K ? nlimk : T.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // loader: thread -> (row, 4 consecutive k) of the slab, for A and for B
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const cplx *pa = T.A + (int64_t)T.arowmap[min(lr, M - 1)] * T.lda;
  const cplx *pb = T.B + (int64_t)T.browmap[min(lr, N - 1)] * T.ldb;
  double2 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + lk + q;
      ra[q] = k < K ? ld2(pa + k) : make_double2(0.0, 0.0);
      rb[q] = k < K ? ld2(pb + k) : make_double2(0.0, 0.0);
    }
  };
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const bool active = wr < M && wc < N;
  bool blk[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) blk[r][c] = wr + 16 * r < M && wc + 16 * c < N;
  // three-product complex form (see gemm_tile): k1 -> cre, k2 -> cim, k3
  d4 cre[2][2], cim[2][2], ck3[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      cre[r][c] = d4{0, 0, 0, 0};
      cim[r][c] = d4{0, 0, 0, 0};
      ck3[r][c] = d4{0, 0, 0, 0};
    }
  load(0);
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();   // the previous slab's MFMA reads are done
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[lk + q][lr ^ GP::swz(lk + q)] = ra[q];
      Bs[lk + q][lr ^ GP::swz(lk + q)] = rb[q];
    }
    __syncthreads();
    if (k0 + 16 < K) load(k0 + 16);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int kx = kk + (lane >> 4);
        double2 a[2], b[2];
        a[0] = As[kx][(wr + (lane & 15)) ^ GP::swz(kx)];
        a[1] = As[kx][(wr + 16 + (lane & 15)) ^ GP::swz(kx)];
        b[0] = Bs[kx][(wc + (lane & 15)) ^ GP::swz(kx)];
        b[1] = Bs[kx][(wc + 16 + (lane & 15)) ^ GP::swz(kx)];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (blk[r][c]) {
              cre[r][c] = GP::mfma(a[r].x + a[r].y, b[c].x, cre[r][c]);
              cim[r][c] = GP::mfma(a[r].x, b[c].y - b[c].x, cim[r][c]);
              ck3[r][c] = GP::mfma(a[r].y, b[c].x + b[c].y, ck3[r][c]);
            }
      }
    }
  }
  if (!active) return;
  const bool acc = coff > 0;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = wr + 16 * r + GP::row(lane, q), j = wc + 16 * c + (lane & 15);
        if (i < M && j < N) {
          cplx *w = T.C + (int64_t)i * T.ldc + j;
          double2 v = make_double2(cre[r][c][q] - ck3[r][c][q], cre[r][c][q] + cim[r][c][q]);
          if (acc) v = cadd(v, ld2(w));
          st2(w, v);
        }
      }
}

// One front of a low-rank sweep subtree (one workgroup): the gradient of its
// pixels, grad_i = scale * Re Rt[i][i] = scale * Re Qt[i][kinv(i)], and the
// Wt of its children in low-rank subtrees, gathered from Rt through their row
// maps (kinv(i): the step whose pivot row is i).
__global__ __launch_bounds__(256) void k_wprop(const WFront *fr, double scale, double *grad) {
  const WFront F = fr[blockIdx.x];
  __shared__ int kinv[MAX_PIVOTS];   // the plan builder rejects larger pivot blocks here
  const int p = F.p, ld = F.p + F.b;
  for (int k = threadIdx.x; k < p; k += blockDim.x) kinv[F.perm[k]] = k;
  __syncthreads();
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const int gi = F.gidx[i];
    if (gi >= 0) grad[gi] = scale * F.Qt[(int64_t)i * ld + kinv[i]].re;
  }
  for (int c = 0; c < F.nch; ++c) {
    const int bc = F.bc[c], ldd = F.pc[c] + bc;
    const int32_t *rm = F.rmap[c];
    cplx *dst = F.dst[c];
    for (int e = threadIdx.x; e < bc * bc; e += blockDim.x) {
      const int y = e / bc, x = e - y * bc;
      const int ry = rm[y], rx = rm[x];
      double2 v;
      if (ry < p) {
        v = rx < p ? ld2(F.Qt + (int64_t)ry * ld + kinv[rx]) : ld2(F.Qt + (int64_t)ry * ld + rx);
        if (rx >= p) v = make_double2(-v.x, -v.y);
      } else {
        const cplx *row = F.Bf + (int64_t)(ry - p) * ld;
        v = rx < p ? ld2(row + kinv[rx]) : ld2(row + rx);
        if (rx < p) v = make_double2(-v.x, -v.y);
      }
      st2(dst + (int64_t)y * ldd + x, v);
    }
  }
}

// grad[g] = scale * (sum of the nblk contraction partials of slot g); the
// partials are block-major, part[b * n + g], so that the threads of a wave
// read consecutive slots
__global__ void k_reduce_partials(const double *part, int nblk, int64_t n, double scale, double *grad) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[(int64_t)b * n + g];
  grad[g] = scale * acc;
}

// ---------------------------------------------------------------------------
// f = sum w |S|^2, dF/dS = w conj(S): block partial sums, then one block.
// ---------------------------------------------------------------------------
__global__ void k_wpow_partial(const double2 *S, const double *w, double2 *G, int64_t n, double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double2 s = S[t];
    double ww = w[t];
    acc += ww * (s.x * s.x + s.y * s.y);
    G[t] = make_double2(ww * s.x, -ww * s.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_wpow_final(const double *part, int n, double *f) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) acc += part[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *f = red[0];
}

// ---------------------------------------------------------------------------
// Beam-splitter figure of merit (Eq. (5)): f = sum (|S|^2 - t)^2 with
// t = t1 where the output order differs from the input order by +-1, else 0;
// dF/dS = 2 (|S|^2 - t) conj(S).  Block partial sums, then k_wpow_final.
// ---------------------------------------------------------------------------
__global__ void k_splitter_partial(const double2 *S, const int32_t *in_ord, const int32_t *out_ord, int n_in,
                                   double t1, double2 *G, int64_t n, double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e / n_in), m = (int)(e - (int64_t)o * n_in);
    const int d = out_ord[o] - in_ord[m];
    const double t = (d == 1 || d == -1) ? t1 : 0.0;
    const double2 v = S[e];
    const double r = v.x * v.x + v.y * v.y - t;
    acc += r * r;
    G[e] = make_double2(2.0 * r * v.x, -2.0 * r * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Grouped objective of the multi-angle splitter: for input a the targets are
// the outputs whose order differs by g * delta, |g| <= gmax; with p = |S|^2
// and mu_a the mean of p over a's targets,
//   f = sum_a sum_t [ -p_ta + (p_ta - mu_a)^2 ],
//   dF/dS_ta = (-1 + 2 (p_ta - mu_a)) conj(S_ta) on the targets, 0 elsewhere.
// k_group_zero clears dF/dS; k_group_partial takes one input column per
// wave at a time, its lanes striding over the outputs (two passes: the mean,
// then f and dF/dS), and sums its block's f into part[]; k_wpow_final adds
// the parts.
// ---------------------------------------------------------------------------
__global__ void k_group_zero(double2 *G, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    G[e] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_group_partial(const double2 *S, const int32_t *in_ord,
                                                      const int32_t *out_ord, int n_in, int n_out, int delta,
                                                      int gmax, double2 *G, double *part) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc = 0.0;   // f over this wave's input columns
  for (int a = blockIdx.x * 4 + wv; a < n_in; a += gridDim.x * 4) {
    const int oa = in_ord[a];
    auto is_target = [&](int t) {
      const int d = out_ord[t] - oa;
      return d % delta == 0 && d <= gmax * delta && -d <= gmax * delta;
    };
    double sum = 0.0;
    int cnt = 0;
    for (int t = lane; t < n_out; t += 64)
      if (is_target(t)) {
        const double2 v = S[(int64_t)t * n_in + a];
        sum += v.x * v.x + v.y * v.y;
        ++cnt;
      }
    for (int off = 32; off > 0; off >>= 1) {
      sum += __shfl_xor(sum, off, 64);
      cnt += __shfl_xor(cnt, off, 64);
    }
    if (cnt > 0) {
      const double mu = sum / cnt;
      double fa = 0.0;
      for (int t = lane; t < n_out; t += 64)
        if (is_target(t)) {
          const double2 v = S[(int64_t)t * n_in + a];
          const double p = v.x * v.x + v.y * v.y, dev = p - mu;
          fa += -p + dev * dev;
          const double df = -1.0 + 2.0 * dev;
          G[(int64_t)t * n_in + a] = make_double2(df * v.x, -df * v.y);
        }
      for (int off = 32; off > 0; off >>= 1) fa += __shfl_xor(fa, off, 64);
      acc += fa;
    }
  }
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// Ridge permittivity from edge positions (grid units along the periodic axis,
// node j = cell [j - 1/2, j + 1/2)); with mirror symmetry the given edges are
// the first half period's and the full list continues with nx - x in
// reverse order.  Ridges are consecutive edge pairs; a cell's permittivity
// is eps_gap + (eps_ridge - eps_gap) * (covered fraction), on every design
// row.  One thread per cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ridge_edge(const double *e, int n, int mirror, int nx, int q) {
  return (!mirror || q < n) ? e[q] : (double)nx - e[2 * n - 1 - q];
}

__global__ void k_ridges_eps(const double *edges, int n, int mirror, int nx, int row0, int nrows, double eps_ridge,
                             double eps_gap, double *eps) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nx) return;
  const int nfull = mirror ? 2 * n : n;
  const double lo = (double)j - 0.5, hi = lo + 1.0;
  double frac = 0.0;
  for (int r = 0; r + 1 < nfull; r += 2) {
    const double a = ridge_edge(edges, n, mirror, nx, r), b = ridge_edge(edges, n, mirror, nx, r + 1);
    for (int sh = -1; sh <= 1; ++sh) {
      const double c = fmin(hi, b + sh * (double)nx) - fmax(lo, a + sh * (double)nx);
      if (c > 0.0) frac += c;
    }
  }
  const double v = eps_gap + (eps_ridge - eps_gap) * frac;
  for (int i = 0; i < nrows; ++i) eps[(int64_t)(row0 + i) * nx + j] = v;
}

// df/dx_k for the free edges: the cell holding an edge changes its covered
// length by -1 (left edge, even place in the full list) or +1 (right edge)
// per unit move; an image edge nx - x moves by -1.  grad_eps: [nrows][nx].
// One workgroup per free edge: the column sums over the design rows.
__device__ double column_sum(const double *g, int nx, int nrows, int j, double *red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nrows; i += blockDim.x) acc += g[(int64_t)i * nx + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(64) void k_ridges_grad(const double *edges, int n, int mirror, int nx, int nrows,
                                                    double eps_ridge, double eps_gap, const double *grad_eps,
                                                    double *grad_edges) {
  __shared__ double red[64];
  const int k = blockIdx.x;
  const double de = eps_ridge - eps_gap;
  const int nfull = mirror ? 2 * n : n;
  auto cell = [&](double x) { int c = (int)floor(x + 0.5) % nx; return c < 0 ? c + nx : c; };
  double g = (k % 2 == 0 ? -de : de) * column_sum(grad_eps, nx, nrows, cell(edges[k]), red);
  if (mirror) {
    const int q = nfull - 1 - k;
    const double sq = q % 2 == 0 ? -de : de;
    g -= sq * column_sum(grad_eps, nx, nrows, cell(ridge_edge(edges, n, mirror, nx, q)), red);
  }
  if (threadIdx.x == 0) grad_edges[k] = g;
}

// ---------------------------------------------------------------------------
// Iterative refinement of the mixed path (FP32 front GEMMs): full-grid
// right-hand sides in elimination order (row e = elimination index of a node,
// `ld` columns), FP64 residuals from the stencil values, and the FP64
// products that turn the refined fields into S and the gradient.
// ---------------------------------------------------------------------------

// Channel matrices of the refined path: Bmat [nx][n_in] = the source row's
// entries of B (-2i sqrt(sin q_a) phi_a(i)) and Cmat [n_out][nx] = the
// projection row's entries of C (sqrt(sin q_b) conj(phi_b(i))).
__global__ void k_channel_matrices(const ChanParams *cp_src, const ChanParams *cp_prj, cplx *Bmat, cplx *Cmat) {
  const Phys &P = cp_src->P;
  const int nx = P.nx, mi = cp_src->m, mo = cp_prj->m;
  const int64_t nb = (int64_t)nx * mi, nc = (int64_t)mo * nx;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nb + nc; t += (int64_t)gridDim.x * blockDim.x) {
    if (t < nb) {
      const int i = (int)(t / mi), a = (int)(t - (int64_t)i * mi);
      const double2 v = channel_value(P, cp_src->orders[a], i, P.eps_src, false);
      st2(Bmat + t, make_double2(2.0 * v.y, -2.0 * v.x));   // times -2i
    } else {
      const int64_t u = t - nb;
      const int b = (int)(u / nx), i = (int)(u - (int64_t)b * nx);
      st2(Cmat + u, channel_value(P, cp_prj->orders[b], i, P.eps_prj, true));
    }
  }
}

// W = r - A X over the whole grid for the first w columns, one wave per node:
// r is zero except on grid row rrow, where r(i, j) = rb[i * ldr + coff + j];
// A X from the five stencil values of the node (A's row) and the fields of
// its neighbours (x periodic; no neighbour past the first and last rows).
// first: X is taken as zero (W = r).  The squared norm of the residual is
// added to *norm2 (a convergence measure only: atomic, order-free).
__global__ __launch_bounds__(256) void k_residual(int nx, int ny, const int32_t *elim, const cplx *Aval,
                                                  const cplx *X, cplx *W, int ld, int w, int rrow, const cplx *rb,
                                                  int ldr, int coff, int first, double *norm2) {
  const int lane = threadIdx.x & 63;
  const int64_t n = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  double acc = 0.0;
  if (n < (int64_t)nx * ny) {
    const int y = (int)(n / nx), x = (int)(n - (int64_t)y * nx);
    const int64_t e = elim[n];
    int64_t nb[5];
    nb[0] = e;
    nb[1] = elim[(int64_t)y * nx + (x == 0 ? nx - 1 : x - 1)];
    nb[2] = elim[(int64_t)y * nx + (x == nx - 1 ? 0 : x + 1)];
    nb[3] = y > 0 ? elim[n - nx] : -1;
    nb[4] = y < ny - 1 ? elim[n + nx] : -1;
    double2 a[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) a[d] = ld2(Aval + n * 5 + d);
    const cplx *rrowp = y == rrow ? rb + (int64_t)x * ldr + coff : nullptr;
    for (int j = lane; j < w; j += 64) {
      double2 v = rrowp ? ld2(rrowp + j) : make_double2(0.0, 0.0);
      if (!first) {
#pragma unroll
        for (int d = 0; d < 5; ++d)
          if (nb[d] >= 0) v = csub(v, cmul(a[d], ld2(X + nb[d] * ld + j)));
      }
      st2(W + e * ld + j, v);
      acc += v.x * v.x + v.y * v.y;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0 && acc != 0.0) atomicAdd(norm2, acc);
}

// X += W (first: X = W) over the first w columns of every row.
__global__ void k_add_fields(cplx *X, const cplx *W, int64_t rows, int ld, int w, int first) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t r = t / w;
  if (r >= rows) return;
  const int64_t o = r * ld + (t - r * w);
  st2(X + o, first ? ld2(W + o) : cadd(ld2(X + o), ld2(W + o)));
}

// Ydes[k][coff + j] = X[erow[k]][j] for the design pixels k (one wave each).
__global__ __launch_bounds__(256) void k_gather_rows(const int32_t *erow, int64_t n, const cplx *X, int ld, int w,
                                                     cplx *Y, int64_t ldy, int coff) {
  const int lane = threadIdx.x & 63;
  const int64_t k = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= n) return;
  const cplx *src = X + (int64_t)erow[k] * ld;
  cplx *dst = Y + k * ldy + coff;
  for (int j = lane; j < w; j += 64) st2(dst + j, ld2(src + j));
}

// grad[k] (+)= scale * Re sum_j Lam[erow[k]][j] Ydes[k][coff + j] over the
// chunk's w columns (one wave per design pixel; the first chunk stores).
__global__ __launch_bounds__(256) void k_contract_rows(const int32_t *erow, int64_t n, const cplx *Lam, int ld, int w,
                                                       const cplx *Y, int64_t ldy, int coff, double scale, int first,
                                                       double *grad) {
  const int lane = threadIdx.x & 63;
  const int64_t k = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= n) return;
  const cplx *l = Lam + (int64_t)erow[k] * ld;
  const cplx *yv = Y + k * ldy + coff;
  double acc = 0.0;
  for (int j = lane; j < w; j += 64) {
    const double2 a = ld2(l + j), b = ld2(yv + j);
    acc += a.x * b.x - a.y * b.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) grad[k] = first ? scale * acc : grad[k] + scale * acc;
}

// Contiguous copies (one block per range).
__global__ void k_copy(const CopyRange *r) {
  const CopyRange c = r[blockIdx.x];
  const double2 *s = reinterpret_cast<const double2 *>(c.src);
  double2 *d = reinterpret_cast<double2 *>(c.dst);
  for (int64_t i = threadIdx.x; i < c.n; i += blockDim.x) d[i] = s[i];
}

// dst (rows x cols, ld ldd) = src^T (src: cols x rows, ld lds), row r of dst
// scaled by 1 / diag[r * ldiag + r] when diag is given: with diag the
// diagonal of U^-1 of a symmetric pivot block this forms U12 = D L21^T from
// L21, without it Z = X12^T.  One workgroup per task, 32 x 32 tiles through
// LDS so that both the reads of src rows and the writes of dst rows are
// coalesced.
__global__ __launch_bounds__(256) void k_transpose_scale(const TransTask *tasks) {
  const TransTask T = tasks[blockIdx.x];
  __shared__ double2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int r0 = 0; r0 < T.rows; r0 += 32)
    for (int c0 = 0; c0 < T.cols; c0 += 32) {
      __syncthreads();   // the previous tile's reads of LDS are done
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + ty + 8 * q, r = r0 + tx;   // src row c, column r
        if (c < T.cols && r < T.rows) tile[ty + 8 * q][tx] = ld2(T.src + (int64_t)c * T.lds + r);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + ty + 8 * q, c = c0 + tx;
        if (r < T.rows && c < T.cols) {
          double2 v = tile[tx][ty + 8 * q];
          if (T.diag) v = cmul(v, cinv(ld2(T.diag + (int64_t)r * T.ldiag + r)));
          st2(T.dst + (int64_t)r * T.ldd + c, v);
        }
      }
    }
}

__global__ void k_fill_double(double *p, int n, double v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// ---------------------------------------------------------------------------
// Parameter-augmented factorization (Eq. (4)): unit entries of the singular
// vectors U (columns) and U^T (rows) in the fronts' augmented panels, and
// Eq. (3) summed per parameter.
// ---------------------------------------------------------------------------
__global__ void k_set_one(cplx *const *p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) st2(p[t], make_double2(1.0, 0.0));
}

// df/dp_k = -2 sum over the columns c of parameter k of sigma_c Re(v_c),
// v_c = sum_m (C A^-1 U)^T dF/dS ... (U^T A^-1 B) of column c; a parameter's
// columns are the range [cbeg[k], cbeg[k + 1]).
__global__ void k_param_sum(const int32_t *cbeg, int np, const double *sigma, const double *v, double *dfdp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  double acc = 0.0;
  for (int c = cbeg[k]; c < cbeg[k + 1]; ++c) acc += sigma[c] * v[c];
  dfdp[k] = -2.0 * acc;
}

// Set (on) or clear the three-product flag of n GEMM tasks (autotuner).
__global__ void k_set_k3(GemmTask *t, int n, int on) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i].flags = on ? (t[i].flags | G_K3) : (t[i].flags & ~G_K3);
}

// ---------------------------------------------------------------------------
// Weighted adjoint source for a dF/dS with few nonzeros per input column
// (such as an objective over a few target orders per input): the columns are
// compacted to (output index, value) lists and V = XC G is formed from them,
// reading each row of XC where the column's nonzeros sit; the same values as
// the dense product (whose other terms are exact zeros).
// ---------------------------------------------------------------------------

// Nonzero count of every column of G (n_out x n_in, row-major); the largest
// goes to *maxnnz.
__global__ __launch_bounds__(256) void k_col_nnz(const double2 *G, int n_out, int n_in, int *nnz, int *maxnnz) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int m = blockIdx.x * 4 + wv; m < n_in; m += gridDim.x * 4) {
    int c = 0;
    for (int b = lane; b < n_out; b += 64) {
      const double2 v = G[(int64_t)b * n_in + m];
      c += (v.x != 0.0 || v.y != 0.0);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) {
      nnz[m] = c;
      atomicMax(maxnnz, c);
    }
  }
}

// The first K nonzeros of every column as (row, value), in row order; unused
// slots hold row 0 and value 0.  One column per wave at a time: each step
// takes 64 consecutive rows, and a lane's slot is the nonzeros before it
// (ballot) after those of the earlier steps.
__global__ __launch_bounds__(256) void k_col_compact(const double2 *G, int n_out, int n_in, int K, int32_t *idx,
                                                    double2 *val) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1;
  for (int m = blockIdx.x * 4 + wv; m < n_in; m += gridDim.x * 4) {
    int c = 0;
    for (int b0 = 0; b0 < n_out && c < K; b0 += 64) {
      const int b = b0 + lane;
      double2 v = make_double2(0.0, 0.0);
      if (b < n_out) v = G[(int64_t)b * n_in + m];
      const bool nz = v.x != 0.0 || v.y != 0.0;
      const unsigned long long mask = __ballot(nz);
      const int slot = c + __popcll(mask & below);
      if (nz && slot < K) {
        idx[(int64_t)m * K + slot] = b;
        val[(int64_t)m * K + slot] = v;
      }
      c += __popcll(mask);
    }
    for (int q = min(c, K) + lane; q < K; q += 64) {
      idx[(int64_t)m * K + q] = 0;
      val[(int64_t)m * K + q] = make_double2(0.0, 0.0);
    }
  }
}

// V[vmap[r]][j] = sum_k XC[r][idx[m][k]] val[m][k], m = coff + j, for the
// chunk's w columns.  A workgroup takes SV_ROWS consecutive rows and 256
// consecutive columns: a thread loads its column's K (row, value) pairs once
// and serves the rows with them; a wave reads consecutive entries of an XC
// row (the target orders of consecutive inputs are consecutive) and writes
// consecutive entries of a V row.
constexpr int SV_ROWS = 8;
template <int SV_KMAX>
__global__ __launch_bounds__(256) void k_sparse_vinit(const double2 *XC, int n_out, int64_t rows,
                                                      const int32_t *vmap, const int32_t *idx, const double2 *val,
                                                      int K, int coff, int w, double2 *V, int ldv) {
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= w) return;
  const int m = coff + j;
  int ik[SV_KMAX];
  double2 gk[SV_KMAX];
#pragma unroll
  for (int k = 0; k < SV_KMAX; ++k)
    if (k < K) {
      ik[k] = idx[(int64_t)m * K + k];
      gk[k] = val[(int64_t)m * K + k];
    }
  const int64_t r0 = (int64_t)blockIdx.x * SV_ROWS;
#pragma unroll
  for (int q = 0; q < SV_ROWS; ++q) {
    const int64_t r = r0 + q;
    if (r >= rows) break;
    const double2 *x = XC + r * n_out;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < SV_KMAX; ++k)
      if (k < K) {
        const double2 a = x[ik[k]];
        acc.x = fma(a.x, gk[k].x, fma(-a.y, gk[k].y, acc.x));
        acc.y = fma(a.x, gk[k].y, fma(a.y, gk[k].x, acc.y));
      }
    V[(int64_t)vmap[r] * ldv + j] = acc;
  }
}

// ---------------------------------------------------------------------------
// Compressed channels (Supplement Sec. 1, this library's reading): the Mx
// extended orders a'_t = a0 + t carry window weights w_t = sin^2(pi (t + 1/2) / Mx);
// column j of the compressed basis on a channel row is
//   sum_t w_t exp(2 pi i a'_t x / nx) exp(-2 pi i t j / Mx) / sqrt(nx),
// localized around x_j = j nx / Mx and truncated to the nodes within
// half_px of x_j (periodic distance).  out (nx x Mx, zeroed beforehand)
// receives the window's entries; conj_all conjugates them (projection rows).
// One thread per (column, node of its window).
// ---------------------------------------------------------------------------
__global__ void k_compress_basis(int nx, int Mx, int a0, double half_px, int lo, int hi, int conj_all, cplx *out) {
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t j = t0 / (hi - lo + 1);
  if (j >= Mx) return;
  const int off = (int)(t0 - j * (hi - lo + 1)) + lo;   // distinct nodes: hi - lo + 1 <= nx
  const double xj = (double)j * nx / Mx;
  int i = (int)floor(xj + 0.5) + off;
  i = ((i % nx) + nx) % nx;
  double d = fabs((double)i - xj);
  d = fmin(d, (double)nx - d);
  if (d > half_px) return;
  double re = 0.0, im = 0.0;
  for (int t = 0; t < Mx; ++t) {
    const double wt = sin(M_PI * (t + 0.5) / Mx);
    const int64_t ai = (((int64_t)(a0 + t) * i) % nx + nx) % nx;
    const int64_t tj = ((int64_t)t * j) % Mx;
    const double ang = 2.0 * M_PI * ((double)ai / nx - (double)tj / Mx);
    double sn, cs;
    sincos(ang, &sn, &cs);
    re += wt * wt * cs;
    im += wt * wt * sn;
  }
  const double sc = 1.0 / sqrt((double)nx);
  st2(out + (int64_t)i * Mx + j, make_double2(re * sc, conj_all ? -im * sc : im * sc));
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_zero(const ZeroRange *r, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(n), dim3(256), 0, s, r);
  return hipGetLastError();
}
hipError_t launch_stencil(const Phys &P, const double *eps, cplx *Aval, int *status, hipStream_t s) {
  int64_t N = (int64_t)P.nx * P.ny;
  hipLaunchKernelGGL(k_stencil, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, P, eps, Aval, status);
  return hipGetLastError();
}
hipError_t launch_scatter_A(const AsmEntry *e, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_A, dim3((n + 255) / 256), dim3(256), 0, s, e, n);
  return hipGetLastError();
}
hipError_t launch_fill_int(int *p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_assemble_panel(const PanelEntry *e, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble_panel, dim3(n), dim3(256), 0, s, e);
  return hipGetLastError();
}
// Largest pivot block of each variant of launch_inverse.
constexpr int kInvCover[N_INV_VARIANTS] = {8 * 2, 8 * 4, 8 * 6, 16 * 4, 32 * 3, 32 * 4};
static_assert(kInvCover[N_INV_VARIANTS - 1] == MAX_PIVOTS, "the largest variant covers exactly MAX_PIVOTS");
int inverse_variant(int p) {
  for (int v = 0; v < N_INV_VARIANTS; ++v)
    if (p >= 1 && p <= kInvCover[v]) return v;
  return -1;
}

// Small blocks (p <= 48, the leaves and short separators) run on one wave:
// the per-step barriers are then free and more fronts fit on a CU.
hipError_t launch_inverse(int variant, const FrontDev *fr, const int32_t *ids, int n, int *status, double *pivq,
                          int sym, hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_lu_inv_reg<8, 8, 2, 2>), dim3(n), dim3(64), 0, s, fr, ids, status, pivq, sym); break;
    case 1: hipLaunchKernelGGL((k_lu_inv_reg<8, 8, 4, 4>), dim3(n), dim3(64), 0, s, fr, ids, status, pivq, sym); break;
    case 2: hipLaunchKernelGGL((k_lu_inv_reg<8, 8, 6, 6>), dim3(n), dim3(64), 0, s, fr, ids, status, pivq, sym); break;
    case 3: hipLaunchKernelGGL((k_lu_inv_reg<16, 16, 4, 4>), dim3(n), dim3(256), 0, s, fr, ids, status, pivq, sym); break;
    case 4: hipLaunchKernelGGL((k_lu_inv_reg<32, 16, 3, 6>), dim3(n), dim3(512), 0, s, fr, ids, status, pivq, sym); break;
    case 5: hipLaunchKernelGGL((k_lu_inv_reg<32, 16, 4, 8>), dim3(n), dim3(512), 0, s, fr, ids, status, pivq, sym); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lowrank_w(const GemmTask *t, int n, int coff, int nlim, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lowrank_w, dim3(n), dim3(256), 0, s, t, coff, nlim);
  return hipGetLastError();
}
hipError_t launch_wprop(const WFront *f, int n, double scale, double *grad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wprop, dim3(n), dim3(256), 0, s, f, scale, grad);
  return hipGetLastError();
}
hipError_t launch_gemm(const GemmTask *t, int n, int coff, int nlim, const cplx *ext, hipStream_t s, bool f32,
                       double *part, int pstride, bool deep, int nthin, int nthin_tri) {
  if (n == 0) return hipSuccess;
  const int nreg = n - nthin;
  if (nreg > 0) {
    if (deep && !f32)
      hipLaunchKernelGGL(k_gemm_k3, dim3(nreg), dim3(256), 0, s, t, coff, nlim, ext, part, pstride);
    else if (f32)
      hipLaunchKernelGGL(k_gemm<true>, dim3(nreg), dim3(256), 0, s, t, coff, nlim, ext, part, pstride);
    else
      hipLaunchKernelGGL(k_gemm<false>, dim3(nreg), dim3(256), 0, s, t, coff, nlim, ext, part, pstride);
  }
  const int nplain = nthin - nthin_tri, ntri = nthin_tri;
  if (nplain > 0) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (f32)
      hipLaunchKernelGGL(k_gemm_thin<true>, dim3(nplain), dim3(256), 0, s, t + nreg, coff, nlim, ext, part, pstride);
    else
      hipLaunchKernelGGL(k_gemm_thin<false>, dim3(nplain), dim3(256), 0, s, t + nreg, coff, nlim, ext, part, pstride);
  }
  if (ntri > 0) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (f32)
      hipLaunchKernelGGL(k_gemm_thin_tri<true>, dim3(ntri), dim3(256), 0, s, t + nreg + nplain, coff, nlim, ext,
                         part, pstride);
    else
      hipLaunchKernelGGL(k_gemm_thin_tri<false>, dim3(ntri), dim3(256), 0, s, t + nreg + nplain, coff, nlim, ext,
                         part, pstride);
  }
  return hipGetLastError();
}

int gemm_kernel_launches(int n, int nthin, int nthin_tri, bool) {
  if (n == 0) return 0;
  return (n - nthin > 0) + (nthin - nthin_tri > 0) + (nthin_tri > 0);
}

// map[r] = base[r] + perm[pidx[r]]: destination rows of a GEMM whose output
// rows follow the pivot permutations computed by the factorization.
__global__ void k_row_map(int32_t *map, const int32_t *base, const int32_t *pidx, const int32_t *perm, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) map[t] = base[t] + perm[pidx[t]];
}

hipError_t launch_row_map(int32_t *map, const int32_t *base, const int32_t *pidx, const int32_t *perm, int64_t n,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, map, base, pidx, perm, n);
  return hipGetLastError();
}

// S = sum over nseg partial products (FP64), one thread per entry.
__global__ void k_sum_partials(const double2 *part, int nseg, int64_t stride, double2 *S, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double2 v = part[t];
  for (int k = 1; k < nseg; ++k) v = cadd(v, part[t + k * stride]);
  S[t] = v;
}

hipError_t launch_sum_partials(const cplx *part, int nseg, int64_t stride, cplx *S, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(part), nseg, stride, reinterpret_cast<double2 *>(S), n);
  return hipGetLastError();
}
hipError_t launch_reduce_partials(const double *part, int nblk, int64_t n, double scale, double *grad,
                                  hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nblk, n, scale,
                     grad);
  return hipGetLastError();
}
hipError_t launch_weighted_power(const cplx *S, const double *w, double *f, cplx *G, int64_t n, double *part,
                                 int npart, hipStream_t s) {
  hipLaunchKernelGGL(k_wpow_partial, dim3(npart), dim3(256), 0, s, reinterpret_cast<const double2 *>(S), w,
                     reinterpret_cast<double2 *>(G), n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wpow_final, dim3(1), dim3(256), 0, s, part, npart, f);
  return hipGetLastError();
}

hipError_t launch_splitter_fom(const cplx *S, const int32_t *in_ord, const int32_t *out_ord, int n_in, int n_out,
                               double t1, double *f, cplx *G, double *part, int npart, hipStream_t s) {
  const int64_t n = (int64_t)n_in * n_out;
  hipLaunchKernelGGL(k_splitter_partial, dim3(npart), dim3(256), 0, s, reinterpret_cast<const double2 *>(S), in_ord,
                     out_ord, n_in, t1, reinterpret_cast<double2 *>(G), n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wpow_final, dim3(1), dim3(256), 0, s, part, npart, f);
  return hipGetLastError();
}
hipError_t launch_group_fom(const cplx *S, const int32_t *in_ord, const int32_t *out_ord, int n_in, int n_out,
                            int delta, int gmax, double *f, cplx *G, double *part, hipStream_t s) {
  const int64_t n = (int64_t)n_in * n_out;
  hipLaunchKernelGGL(k_group_zero, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<double2 *>(G), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = std::min(1024, (n_in + 3) / 4);   // (part holds 1024 blocks' sums)
  hipLaunchKernelGGL(k_group_partial, dim3(nb), dim3(256), 0, s, reinterpret_cast<const double2 *>(S), in_ord,
                     out_ord, n_in, n_out, delta, gmax, reinterpret_cast<double2 *>(G), part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wpow_final, dim3(1), dim3(256), 0, s, part, nb, f);
  return hipGetLastError();
}
hipError_t launch_ridges_eps(const double *edges, int n, int mirror, int nx, int row0, int nrows, double eps_ridge,
                             double eps_gap, double *eps, hipStream_t s) {
  hipLaunchKernelGGL(k_ridges_eps, dim3((nx + 255) / 256), dim3(256), 0, s, edges, n, mirror, nx, row0, nrows,
                     eps_ridge, eps_gap, eps);
  return hipGetLastError();
}
hipError_t launch_ridges_grad(const double *edges, int n, int mirror, int nx, int nrows, double eps_ridge,
                              double eps_gap, const double *grad_eps, double *grad_edges, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ridges_grad, dim3(n), dim3(64), 0, s, edges, n, mirror, nx, nrows, eps_ridge, eps_gap,
                     grad_eps, grad_edges);
  return hipGetLastError();
}

hipError_t launch_channel_matrices(const ChanParams *cp_src, const ChanParams *cp_prj, cplx *Bmat, cplx *Cmat,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_channel_matrices, dim3(2048), dim3(256), 0, s, cp_src, cp_prj, Bmat, Cmat);
  return hipGetLastError();
}
hipError_t launch_residual(int nx, int ny, const int32_t *elim, const cplx *Aval, const cplx *X, cplx *W, int ld,
                           int w, int rrow, const cplx *rb, int ldr, int coff, bool first, double *norm2,
                           hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, nx, ny, elim, Aval, X, W, ld, w,
                     rrow, rb, ldr, coff, first ? 1 : 0, norm2);
  return hipGetLastError();
}
hipError_t launch_add_fields(cplx *X, const cplx *W, int64_t rows, int ld, int w, bool first, hipStream_t s) {
  const int64_t n = rows * w;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_fields, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, W, rows, ld, w,
                     first ? 1 : 0);
  return hipGetLastError();
}
hipError_t launch_gather_rows(const int32_t *erow, int64_t n, const cplx *X, int ld, int w, cplx *Y, int64_t ldy,
                              int coff, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, erow, n, X, ld, w, Y, ldy, coff);
  return hipGetLastError();
}
hipError_t launch_contract_rows(const int32_t *erow, int64_t n, const cplx *Lam, int ld, int w, const cplx *Y,
                                int64_t ldy, int coff, double scale, bool first, double *grad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_contract_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, erow, n, Lam, ld, w, Y, ldy,
                     coff, scale, first ? 1 : 0, grad);
  return hipGetLastError();
}
hipError_t launch_transpose_scale(const TransTask *t, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_scale, dim3(n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_copy(const CopyRange *r, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(n), dim3(256), 0, s, r);
  return hipGetLastError();
}
hipError_t launch_fill_double(double *p, int n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_double, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_set_one(cplx *const *p, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_one, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_param_sum(const int32_t *cbeg, int np, const double *sigma, const double *v, double *dfdp,
                            hipStream_t s) {
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_param_sum, dim3((np + 255) / 256), dim3(256), 0, s, cbeg, np, sigma, v, dfdp);
  return hipGetLastError();
}

hipError_t launch_zero_flat(cplx *p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_zero, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<double2 *>(p), n);
  return hipGetLastError();
}

hipError_t launch_set_k3(GemmTask *t, int n, bool on, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_k3, dim3((n + 255) / 256), dim3(256), 0, s, t, n, on ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_col_nnz(const cplx *G, int n_out, int n_in, int *nnz, int *maxnnz, hipStream_t s) {
  // one column per wave (4 per workgroup), grid-strided
  hipLaunchKernelGGL(k_col_nnz, dim3(std::min(65535, (n_in + 3) / 4)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(G), n_out, n_in, nnz, maxnnz);
  return hipGetLastError();
}
hipError_t launch_col_compact(const cplx *G, int n_out, int n_in, int K, int32_t *idx, cplx *val, hipStream_t s) {
  hipLaunchKernelGGL(k_col_compact, dim3(std::min(65535, (n_in + 3) / 4)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(G), n_out, n_in, K, idx, reinterpret_cast<double2 *>(val));
  return hipGetLastError();
}
hipError_t launch_channel_amp(const ChanParams *cp, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_channel_amp, dim3((n + 255) / 256), dim3(256), 0, s, cp, n);
  return hipGetLastError();
}

hipError_t launch_sparse_vinit(const cplx *XC, int n_out, int64_t rows, const int32_t *vmap, const int32_t *idx,
                               const cplx *val, int K, int coff, int w, cplx *V, int ldv, hipStream_t s) {
  if (rows == 0 || w == 0) return hipSuccess;
  if (K < 1 || K > 32) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + SV_ROWS - 1) / SV_ROWS), (unsigned)((w + 255) / 256));
  // (the column's list lives in registers: size the kernel to K)
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, reinterpret_cast<const double2 *>(XC), n_out, rows, vmap, idx,
                       reinterpret_cast<const double2 *>(val), K, coff, w, reinterpret_cast<double2 *>(V), ldv);
  };
  if (K <= 8) go(k_sparse_vinit<8>);
  else if (K <= 16) go(k_sparse_vinit<16>);
  else go(k_sparse_vinit<32>);
  return hipGetLastError();
}

hipError_t launch_compress_basis(int nx, int Mx, int a0, double half_px, bool conj_all, cplx *out, hipStream_t s) {
  const double reach = std::ceil(half_px) + 1.0;
  const int lo = -(int)std::min<double>(reach, (double)((nx - 1) / 2)), hi = (int)std::min<double>(reach, nx / 2);
  const int64_t n = (int64_t)Mx * (hi - lo + 1);
  hipLaunchKernelGGL(k_compress_basis, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nx, Mx, a0, half_px, lo, hi,
                     conj_all ? 1 : 0, out);
  return hipGetLastError();
}

}  // namespace apf
