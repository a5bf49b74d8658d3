// Kernels of the system matrix-vector product (eq. (7)-(8)) and its driver.
//
//   e = Z H,  g = M H (M = Y_eq Z, eq. (6)),  j = H - g (eq. (2)),  q = B c0rho
//   a = L_A j,  phi = L_phi q   (AIM, eq. (11): L_NR + W H P; or dense)
//   y1 = j k0 a + D^T phi + I_x e / eta0,   y2 = F D j + j k0 c0rho
//
// Precision: FP64 (internal blocks as hi + lo complex64, everything else
// complex128) or MIXED (hi complex64 blocks, FP32 accumulation, complex64 FFT,
// near field and vectors).  The ABI vectors are always complex128.
#include "ctx.hpp"

namespace slim {

namespace {

template <class T> struct C2 { T x, y; };
template <class T> __device__ __forceinline__ C2<T> cz() { return {T(0), T(0)}; }

template <bool F64> struct P;
template <> struct P<true> { using T = double; };
template <> struct P<false> { using T = float; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Casts
// ---------------------------------------------------------------------------
__global__ void k_c128_to_c64(const double2* in, float2* out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(float(in[i].x), float(in[i].y));
}
__global__ void k_c64_to_c128(const float2* in, double2* out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2(double(in[i].x), double(in[i].y));
}

// ---------------------------------------------------------------------------
// Build helpers
// ---------------------------------------------------------------------------
// Column-major complex128 Z and M (n x n) -> rows of the stacked row-major block
// [Z; M] with leading dimension ld, split into hi = fl32(v), lo = fl32(v - hi).
__global__ void k_pack_block(const double2* Z, const double2* M, int n, int ld, float2* hi, float2* lo) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t tot = int64_t(2 * n) * ld;
  if (i >= tot) return;
  const int row = int(i / ld), col = int(i % ld);
  double2 v = make_double2(0.0, 0.0);
  if (col < n) v = row < n ? Z[row + int64_t(col) * n] : M[(row - n) + int64_t(col) * n];
  float2 h = make_float2(float(v.x), float(v.y));
  hi[i] = h;
  lo[i] = make_float2(float(v.x - double(h.x)), float(v.y - double(h.y)));
}

__global__ void k_pack_dense(const double2* A, int64_t n, float2* hi, float2* lo) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v = A[i];
  float2 h = make_float2(float(v.x), float(v.y));
  hi[i] = h;
  lo[i] = make_float2(float(v.x - double(h.x)), float(v.y - double(h.y)));
}

// B (column-major n x n, local RWG indices) += half * I_x
__global__ void k_add_ix(double2* B, const int32_t* col, const double* val, int e0, int n, double half) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  for (int q = 0; q < 4; ++q) {
    const int c = col[4 * (e0 + m) + q];
    if (c < 0) continue;
    double2& d = B[m + int64_t(c - e0) * n];
    d.x += half * val[4 * (e0 + m) + q];
  }
}

__global__ void k_scale(double2* M, int64_t n, double fr, double fi) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v = M[i];
  M[i] = make_double2(v.x * fr - v.y * fi, v.x * fi + v.y * fr);
}

// Back substitution on one diagonal block of an upper-triangular factor:
// X[i0 : i0+nb, c] = U[i0 : i0+nb, i0 : i0+nb]^{-1} X[i0 : i0+nb, c] for every column c
// (one thread per column, the block in LDS).  Together with GEMM updates of the rows
// above it this is the blocked triangular solve without diagonal-block inversion,
// which stays backward stable for factors whose pivots span many decades.
constexpr int kUB = 32;
__global__ void __launch_bounds__(256) k_usolve_block(const double2* U, int64_t ld, int i0, int nb, double2* X,
                                                     int64_t ldx, int nrhs) {
  __shared__ double2 blk[kUB][kUB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int r = e % nb, cc = e / nb;
    blk[r][cc] = U[(i0 + r) + int64_t(i0 + cc) * ld];
  }
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nrhs) return;
  double2 x[kUB];
#pragma unroll
  for (int i = 0; i < kUB; ++i) x[i] = i < nb ? X[(i0 + i) + int64_t(c) * ldx] : make_double2(0.0, 0.0);
#pragma unroll
  for (int i = kUB - 1; i >= 0; --i) {
    if (i >= nb) continue;
    double2 acc = x[i];
#pragma unroll
    for (int j = i + 1; j < kUB; ++j) {
      if (j >= nb) continue;
      const double2 u = blk[i][j];
      acc.x -= u.x * x[j].x - u.y * x[j].y;
      acc.y -= u.x * x[j].y + u.y * x[j].x;
    }
    const double2 d = blk[i][i];
    const double den = d.x * d.x + d.y * d.y;
    x[i] = make_double2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den);
  }
#pragma unroll
  for (int i = 0; i < kUB; ++i)
    if (i < nb) X[(i0 + i) + int64_t(c) * ldx] = x[i];
}

// ---------------------------------------------------------------------------
// A1 + A2: persistent internal GEMV over the slot queues, fused epilogue.
// Each workgroup is one slot; it walks its tiles in order.  A wave takes eight
// consecutive rows at a time and streams them with 16-byte non-temporal loads
// (two complex per lane, two 128-column chunks per iteration: 16 loads in
// flight per lane), sharing the H loads (L2-resident) between the eight rows.
// ---------------------------------------------------------------------------
struct BlockDev { int64_t off; int32_t n; int32_t e0; };

typedef float f4v __attribute__((ext_vector_type(4)));
// 16-byte streaming load of two complex64 values, marked non-temporal (read once)
__device__ __forceinline__ float4 ntload(const float2* p) {
  const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

template <bool F64>
__global__ void __launch_bounds__(256) k_internal(const float2* __restrict__ hi, const float2* __restrict__ lo,
                                                  const BlockDev* __restrict__ blocks, const int4* __restrict__ tiles,
                                                  const int32_t* __restrict__ slot_start, const void* __restrict__ Hv,
                                                  void* __restrict__ ev, void* __restrict__ jv, void* __restrict__ gv,
                                                  unsigned long long* __restrict__ stamps) {
  using T = typename P<F64>::T;
  constexpr int RW = F64 ? 4 : 8;    // rows per wave per sweep (hi + lo doubles the loads in FP64)
  const C2<T>* H = reinterpret_cast<const C2<T>*>(Hv);
  C2<T>* e = reinterpret_cast<C2<T>*>(ev);
  C2<T>* jo = reinterpret_cast<C2<T>*>(jv);
  C2<T>* go = reinterpret_cast<C2<T>*>(gv);
  const int slot = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int ti = slot_start[slot]; ti < slot_start[slot + 1]; ++ti) {
    const int4 tl = tiles[ti];        // block, row0, rows, slot
    unsigned long long t_start = 0;
    if (stamps && threadIdx.x == 0) t_start = wall_clock64();
    const BlockDev B = blocks[tl.x];
    const int n = B.n, ld = (n + 1) & ~1;
    const C2<T>* Hs = H + B.e0;
    const int rend = tl.y + tl.z;
    for (int r0 = tl.y + RW * wave; r0 < rend; r0 += 4 * RW) {
      T ar[RW], ai[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) { ar[q] = 0; ai[q] = 0; }
      const int nr = min(RW, rend - r0);
      const int64_t base = B.off + int64_t(r0) * ld;
      // two column chunks of 128 per iteration: 2 x RW 16-byte loads in flight per lane
      for (int col = 2 * lane; col < ld; col += 256) {
        const int col2 = col + 128;
        C2<T> h0 = cz<T>(), h1 = cz<T>(), h2 = cz<T>(), h3 = cz<T>();
        if (col < n) h0 = Hs[col];
        if (col + 1 < n) h1 = Hs[col + 1];
        if (col2 < n) h2 = Hs[col2];
        if (col2 + 1 < n) h3 = Hs[col2 + 1];
        float4 a[RW], b[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
          b[q] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (q < nr) {
            a[q] = ntload(hi + base + int64_t(q) * ld + col);
            if (col2 < ld)
              b[q] = ntload(hi + base + int64_t(q) * ld + col2);
          }
        }
        float4 al[RW], bl[RW];
        if (F64) {
#pragma unroll
          for (int q = 0; q < RW; ++q) {
            al[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            bl[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < nr) {
              al[q] = ntload(lo + base + int64_t(q) * ld + col);
              if (col2 < ld)
                bl[q] = ntload(lo + base + int64_t(q) * ld + col2);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          T a0r = a[q].x, a0i = a[q].y, a1r = a[q].z, a1i = a[q].w;
          T b0r = b[q].x, b0i = b[q].y, b1r = b[q].z, b1i = b[q].w;
          if (F64) {
            a0r += T(al[q].x); a0i += T(al[q].y); a1r += T(al[q].z); a1i += T(al[q].w);
            b0r += T(bl[q].x); b0i += T(bl[q].y); b1r += T(bl[q].z); b1i += T(bl[q].w);
          }
          ar[q] += a0r * h0.x - a0i * h0.y + a1r * h1.x - a1i * h1.y + b0r * h2.x - b0i * h2.y + b1r * h3.x - b1i * h3.y;
          ai[q] += a0r * h0.y + a0i * h0.x + a1r * h1.y + a1i * h1.x + b0r * h2.y + b0i * h2.x + b1r * h3.y + b1i * h3.x;
        }
      }
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        T sr = wave_sum(ar[q]), si = wave_sum(ai[q]);
        if (lane == 0 && q < nr) {
          const int row = r0 + q;
          if (row < n) {
            e[B.e0 + row] = {sr, si};
          } else {
            const int k = row - n;
            const C2<T> h = Hs[k];
            jo[B.e0 + k] = {h.x - sr, h.y - si};     // j = H - M H
            if (go) go[B.e0 + k] = {sr, si};
          }
        }
      }
    }
    if (stamps) {
      __syncthreads();
      if (threadIdx.x == 0) {
        stamps[2 * ti] = t_start;
        stamps[2 * ti + 1] = wall_clock64();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// A3: projection P as an atomic-free gather over occupied grid nodes.
// RWG list: S_c(node) = sum w_c j_n (c = x, y, z); pulse list: S_rho = sum (w A_t) c0rho_t.
// ---------------------------------------------------------------------------
template <bool F64>
__device__ __forceinline__ typename P<F64>::T group_sum8(typename P<F64>::T v) {
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) v += __shfl_xor(v, off, 8);
  return v;
}

// Eight lanes per occupied node stride its (basis, weight) list, so the list is
// read in contiguous runs; the partial sums meet through lane shuffles.
template <bool F64>
__global__ void __launch_bounds__(256) k_project(const int32_t* pe_node, const int32_t* pe_ptr, const int32_t* pe_idx,
                                                 const void* pe_w, int64_t n_pe, const int32_t* pt_node,
                                                 const int32_t* pt_ptr, const int32_t* pt_idx, const void* pt_w,
                                                 int64_t n_pt, const void* jv, const void* rhov, void* octv, int64_t N3) {
  using T = typename P<F64>::T;
  const T* we = reinterpret_cast<const T*>(pe_w);
  const T* wt = reinterpret_cast<const T*>(pt_w);
  const C2<T>* j = reinterpret_cast<const C2<T>*>(jv);
  const C2<T>* rho = reinterpret_cast<const C2<T>*>(rhov);
  C2<T>* oct = reinterpret_cast<C2<T>*>(octv);
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  if (i < n_pe) {
    T sx0 = 0, sx1 = 0, sy0 = 0, sy1 = 0, sz0 = 0, sz1 = 0;
    for (int z = pe_ptr[i] + sub; z < pe_ptr[i + 1]; z += 8) {
      const C2<T> v = j[pe_idx[z]];
      const T w0 = we[3 * int64_t(z)], w1 = we[3 * int64_t(z) + 1], w2 = we[3 * int64_t(z) + 2];
      sx0 += w0 * v.x; sx1 += w0 * v.y;
      sy0 += w1 * v.x; sy1 += w1 * v.y;
      sz0 += w2 * v.x; sz1 += w2 * v.y;
    }
    sx0 = group_sum8<F64>(sx0); sx1 = group_sum8<F64>(sx1);
    sy0 = group_sum8<F64>(sy0); sy1 = group_sum8<F64>(sy1);
    sz0 = group_sum8<F64>(sz0); sz1 = group_sum8<F64>(sz1);
    if (sub == 0) {
      const int64_t node = pe_node[i];
      oct[node] = {sx0, sx1};
      oct[N3 + node] = {sy0, sy1};
      oct[2 * N3 + node] = {sz0, sz1};
    }
  } else if (i < n_pe + n_pt) {
    const int64_t k = i - n_pe;
    T s0 = 0, s1 = 0;
    for (int z = pt_ptr[k] + sub; z < pt_ptr[k + 1]; z += 8) {
      const C2<T> v = rho[pt_idx[z]];
      s0 += wt[z] * v.x;
      s1 += wt[z] * v.y;
    }
    s0 = group_sum8<F64>(s0);
    s1 = group_sum8<F64>(s1);
    if (sub == 0) oct[3 * N3 + pt_node[k]] = {s0, s1};
  }
}

// ---------------------------------------------------------------------------
// A5 + A6 for pulses: phi_t = W_rho Phi_rho + L_phi,NR (B c0rho); one wave per row.
// ---------------------------------------------------------------------------
template <bool F64>
__global__ void __launch_bounds__(256) k_phi(const int32_t* wt_base, const void* wt_w, const void* octv, int64_t N3,
                                             int Nx, int NxNy, const int64_t* ptr, const int32_t* col,
                                             const void* valv, const void* rhov, void* phiv, int64_t n_t) {
  using T = typename P<F64>::T;
  const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n_t) return;
  const T* w = reinterpret_cast<const T*>(wt_w);
  const C2<T>* Phi = reinterpret_cast<const C2<T>*>(octv) + 3 * N3;
  const C2<T>* val = reinterpret_cast<const C2<T>*>(valv);
  const C2<T>* rho = reinterpret_cast<const C2<T>*>(rhov);
  T sr = 0, si = 0;
  if (lane < 27) {
    const int64_t node = wt_base[t] + (lane % 3) + Nx * ((lane / 3) % 3) + int64_t(NxNy) * (lane / 9);
    const T wv = w[27 * t + lane];
    sr = wv * Phi[node].x;
    si = wv * Phi[node].y;
  }
  const int64_t zend = ptr[t + 1];
  for (int64_t z = ptr[t] + lane; z < zend; z += 128) {
    const bool two = z + 64 < zend;
    const int c0 = col[z], c1 = two ? col[z + 64] : c0;
    const C2<T> a0 = val[z], a1 = two ? val[z + 64] : C2<T>{T(0), T(0)};
    const C2<T> b0 = rho[c0], b1 = rho[c1];
    sr += a0.x * b0.x - a0.y * b0.y + a1.x * b1.x - a1.y * b1.y;
    si += a0.x * b0.y + a0.y * b0.x + a1.x * b1.y + a1.y * b1.x;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) reinterpret_cast<C2<T>*>(phiv)[t] = {sr, si};
}

// ---------------------------------------------------------------------------
// A5 + A6 + A7 for RWG rows: a = W_A Phi + L_A,NR j;
// y1 = j k0 a + l (phi[T+] - phi[T-]) + I_x e / eta0  (written as complex128).
// ---------------------------------------------------------------------------
template <bool F64, bool AIM>
__global__ void __launch_bounds__(256) k_rows_A(const int32_t* we_base, const void* we_w, const void* octv, int64_t N3,
                                                int Nx, int NxNy, const int64_t* ptr, const int32_t* col,
                                                const void* valv, const void* jv, const void* a_dense,
                                                const void* phiv, const void* ev, const int32_t* tplus,
                                                const int32_t* tminus, const double* len, const int32_t* ix_col,
                                                const double* ix_val, double k0, double inv_eta0, void* av,
                                                double2* y, int64_t n_e) {
  using T = typename P<F64>::T;
  const int64_t m = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= n_e) return;
  T sr = 0, si = 0;
  if (AIM) {
    const T* w = reinterpret_cast<const T*>(we_w) + 81 * m;
    const C2<T>* Phi = reinterpret_cast<const C2<T>*>(octv);
    if (lane < 27) {
      const int64_t node = we_base[m] + (lane % 3) + Nx * ((lane / 3) % 3) + int64_t(NxNy) * (lane / 9);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const C2<T> p = Phi[c * N3 + node];
        sr += w[c * 27 + lane] * p.x;
        si += w[c * 27 + lane] * p.y;
      }
    }
    const C2<T>* val = reinterpret_cast<const C2<T>*>(valv);
    const C2<T>* j = reinterpret_cast<const C2<T>*>(jv);
    // two entries per lane per trip: both column loads, then both gathers, are in flight together
    const int64_t zend = ptr[m + 1];
    for (int64_t z = ptr[m] + lane; z < zend; z += 128) {
      const bool two = z + 64 < zend;
      const int c0 = col[z], c1 = two ? col[z + 64] : c0;
      const C2<T> a0 = val[z], a1 = two ? val[z + 64] : C2<T>{T(0), T(0)};
      const C2<T> b0 = j[c0], b1 = j[c1];
      sr += a0.x * b0.x - a0.y * b0.y + a1.x * b1.x - a1.y * b1.y;
      si += a0.x * b0.y + a0.y * b0.x + a1.x * b1.y + a1.y * b1.x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
  } else if (lane == 0) {
    const C2<T> a = reinterpret_cast<const C2<T>*>(a_dense)[m];
    sr = a.x;
    si = a.y;
  }
  if (lane == 0) {
    const C2<T>* phi = reinterpret_cast<const C2<T>*>(phiv);
    const C2<T>* e = reinterpret_cast<const C2<T>*>(ev);
    if (AIM) reinterpret_cast<C2<T>*>(av)[m] = {sr, si};
    const double l = len[m];
    const C2<T> pp = phi[tplus[m]], pm = phi[tminus[m]];
    double yr = -k0 * double(si) + l * (double(pp.x) - double(pm.x));
    double yi = k0 * double(sr) + l * (double(pp.y) - double(pm.y));
    for (int q = 0; q < 4; ++q) {
      const int c = ix_col[4 * m + q];
      if (c < 0) continue;
      const C2<T> ec = e[c];
      yr += inv_eta0 * ix_val[4 * m + q] * double(ec.x);
      yi += inv_eta0 * ix_val[4 * m + q] * double(ec.y);
    }
    y[m] = make_double2(yr, yi);
  }
}

// y2 = F D j + j k0 c0rho = -(1/A_t) sum_i s_i l_i j_i + j k0 c0rho_t
template <bool F64>
__global__ void k_rows_T(const int32_t* tri_edge, const int8_t* tri_sign, const double* len, const double* area,
                         const void* jv, const void* rhov, double k0, double2* y2, int64_t n_t) {
  using T = typename P<F64>::T;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  const C2<T>* j = reinterpret_cast<const C2<T>*>(jv);
  const C2<T> r = reinterpret_cast<const C2<T>*>(rhov)[t];
  double dr = 0.0, di = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int n = tri_edge[3 * t + i];
    const double d = tri_sign[3 * t + i] * len[n];
    dr += d * double(j[n].x);
    di += d * double(j[n].y);
  }
  const double ia = 1.0 / area[t];
  y2[t] = make_double2(-ia * dr - k0 * double(r.y), -ia * di + k0 * double(r.x));
}

// Dense row-major GEMV (plain mode): out = A v, A as hi (+ lo), one wave per row.
template <bool F64>
__global__ void __launch_bounds__(256) k_dense_gemv(const float2* hi, const float2* lo, int64_t n, const void* vv,
                                                    const double* colscale, void* outv) {
  using T = typename P<F64>::T;
  const int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const C2<T>* v = reinterpret_cast<const C2<T>*>(vv);
  T sr = 0, si = 0;
  for (int64_t c = lane; c < n; c += 64) {
    float2 a = hi[r * n + c];
    T ar = a.x, ai = a.y;
    if (F64) { float2 b = lo[r * n + c]; ar += T(b.x); ai += T(b.y); }
    C2<T> x = v[c];
    if (colscale) { x.x *= T(colscale[c]); x.y *= T(colscale[c]); }
    sr += ar * x.x - ai * x.y;
    si += ar * x.y + ai * x.x;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) reinterpret_cast<C2<T>*>(outv)[r] = {sr, si};
}

template <bool F64>
__global__ void k_copy_out(const void* in, double2* out, int64_t n) {
  using T = typename P<F64>::T;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const C2<T> v = reinterpret_cast<const C2<T>*>(in)[i];
  out[i] = make_double2(double(v.x), double(v.y));
}

template <bool F64>
void internal_launch(Ctx& c, const void* H, void* e, void* j, void* g, hipStream_t s) {
  unsigned long long* st = c.record ? c.d_stamps.as<unsigned long long>() : nullptr;
  hipLaunchKernelGGL(k_internal<F64>, dim3(unsigned(c.slots)), dim3(256), 0, s, c.d_hi.as<float2>(),
                     c.d_lo.as<float2>(), c.d_blocks.as<BlockDev>(), c.d_tiles.as<int4>(),
                     c.d_slot_start.as<int32_t>(), H, e, j, g, st);
  SLIM_HIP(hipGetLastError());
}

template <bool F64>
void matvec_t(Ctx& c, const void* x, void* y, void* e_out, void* g_out, void* a_out, void* phi_out, hipStream_t s) {
  const RWGTable& r = c.rwg;
  const int64_t ne = r.n_e, nt = r.n_t, nsys = ne + nt;
  const size_t es = F64 ? 16 : 8;
  const void* X = x;
  if (!F64) {
    hipLaunchKernelGGL(k_c128_to_c64, dim3(nblk(nsys)), dim3(256), 0, s, reinterpret_cast<const double2*>(x),
                       c.d_x64.as<float2>(), nsys);
    SLIM_HIP(hipGetLastError());
    X = c.d_x64.p;
  }
  const char* Xc = reinterpret_cast<const char*>(X);
  const void* rho = Xc + ne * es;
  double2* Y = reinterpret_cast<double2*>(y);
  if (c.prof_on) c.prof_calls++;
  auto mark = [&](int st) { if (c.prof_on) c.prof_mark(st, s); };
  const double inv_eta0 = 1.0 / eta0();
  // The pulse path (projection of B c0rho, its convolution, W and L_phi,NR) does
  // not depend on the internal blocks: without per-stage timing it runs on a
  // second stream, concurrently with them, and joins before the RWG rows.
  const bool aim = !c.plain;
  const bool overlap = aim && !c.prof_on && c.s_phi;
  const int64_t N3 = aim ? c.grid.nodes() : 0;
  void* oct_in = F64 ? c.d_oct_in.p : c.d_oct_in32.p;
  const int Nx = c.grid.N[0], NxNy = c.grid.N[0] * c.grid.N[1];
  auto pulse_path = [&](hipStream_t st) {
    hipLaunchKernelGGL(k_project<F64>, dim3(nblk(8 * c.n_pt_nodes)), dim3(256), 0, st, nullptr, nullptr, nullptr, nullptr,
                       int64_t(0), c.d_pt_node.as<int32_t>(), c.d_pt_ptr.as<int32_t>(), c.d_pt_idx.as<int32_t>(),
                       F64 ? c.d_pt_w64.p : c.d_pt_w32.p, c.n_pt_nodes, nullptr, rho, oct_in, N3);
    SLIM_HIP(hipGetLastError());
    aim_convolve(c, F64, 1, st, 3, c.layered);
    hipLaunchKernelGGL(k_phi<F64>, dim3(nblk(nt, 4)), dim3(256), 0, st, c.d_wt_base.as<int32_t>(),
                       F64 ? c.d_wt_w64.p : c.d_wt_w32.p, c.d_oct_out.p, N3, Nx, NxNy, c.d_nP_ptr.as<int64_t>(),
                       c.d_nP_col.as<int32_t>(), F64 ? c.d_nP_v128.p : c.d_nP_v64.p, rho, c.d_phi.p, nt);
    SLIM_HIP(hipGetLastError());
  };
  if (overlap) {
    SLIM_HIP(hipEventRecord(c.ev_fork, s));
    SLIM_HIP(hipStreamWaitEvent(c.s_phi, c.ev_fork, 0));
    pulse_path(c.s_phi);
    SLIM_HIP(hipEventRecord(c.ev_join, c.s_phi));
  }
  // A1 + A2
  mark(0);
  internal_launch<F64>(c, X, c.d_e.p, c.d_j.p, g_out ? c.d_g.p : nullptr, s);
  mark(0);
  if (c.plain) {
    hipLaunchKernelGGL(k_dense_gemv<F64>, dim3(nblk(nt, 4)), dim3(256), 0, s, c.d_Lphi_hi.as<float2>(),
                       c.d_Lphi_lo.as<float2>(), nt, rho, c.d_area.as<double>(), c.d_phi.p);
    hipLaunchKernelGGL(k_dense_gemv<F64>, dim3(nblk(ne, 4)), dim3(256), 0, s, c.d_LA_hi.as<float2>(),
                       c.d_LA_lo.as<float2>(), ne, c.d_j.p, nullptr, c.d_a.p);
    SLIM_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_rows_A<F64, false>), dim3(nblk(ne, 4)), dim3(256), 0, s, nullptr, nullptr, nullptr,
                       int64_t(0), 0, 0, nullptr, nullptr, nullptr, nullptr, c.d_a.p, c.d_phi.p, c.d_e.p,
                       c.d_tplus.as<int32_t>(), c.d_tminus.as<int32_t>(), c.d_len.as<double>(),
                       c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), c.k0, inv_eta0, nullptr, Y, ne);
  } else {
    mark(1);
    hipLaunchKernelGGL(k_project<F64>, dim3(nblk(8 * (c.n_pe_nodes + (overlap ? 0 : c.n_pt_nodes)))), dim3(256), 0, s,
                       c.d_pe_node.as<int32_t>(), c.d_pe_ptr.as<int32_t>(), c.d_pe_idx.as<int32_t>(),
                       F64 ? c.d_pe_w64.p : c.d_pe_w32.p, c.n_pe_nodes, c.d_pt_node.as<int32_t>(),
                       c.d_pt_ptr.as<int32_t>(), c.d_pt_idx.as<int32_t>(), F64 ? c.d_pt_w64.p : c.d_pt_w32.p,
                       overlap ? int64_t(0) : c.n_pt_nodes, c.d_j.p, rho, oct_in, N3);
    SLIM_HIP(hipGetLastError());
    mark(1);
    mark(2);
    aim_convolve(c, F64, overlap ? 3 : 4, s, 0, c.layered);
    mark(2);
    mark(3);
    if (overlap) {
      SLIM_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
    } else {
      hipLaunchKernelGGL(k_phi<F64>, dim3(nblk(nt, 4)), dim3(256), 0, s, c.d_wt_base.as<int32_t>(),
                         F64 ? c.d_wt_w64.p : c.d_wt_w32.p, c.d_oct_out.p, N3, Nx, NxNy, c.d_nP_ptr.as<int64_t>(),
                         c.d_nP_col.as<int32_t>(), F64 ? c.d_nP_v128.p : c.d_nP_v64.p, rho, c.d_phi.p, nt);
      SLIM_HIP(hipGetLastError());
    }
    mark(3);
    mark(4);
    hipLaunchKernelGGL((k_rows_A<F64, true>), dim3(nblk(ne, 4)), dim3(256), 0, s, c.d_we_base.as<int32_t>(),
                       F64 ? c.d_we_w64.p : c.d_we_w32.p, c.d_oct_out.p, N3, Nx, NxNy, c.d_nA_ptr.as<int64_t>(),
                       c.d_nA_col.as<int32_t>(), F64 ? c.d_nA_v128.p : c.d_nA_v64.p, c.d_j.p, nullptr, c.d_phi.p,
                       c.d_e.p, c.d_tplus.as<int32_t>(), c.d_tminus.as<int32_t>(), c.d_len.as<double>(),
                       c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), c.k0, inv_eta0, c.d_a.p, Y, ne);
    mark(4);
  }
  SLIM_HIP(hipGetLastError());
  mark(5);
  hipLaunchKernelGGL(k_rows_T<F64>, dim3(nblk(nt)), dim3(256), 0, s, c.d_tri_edge.as<int32_t>(),
                     c.d_tri_sign.as<int8_t>(), c.d_len.as<double>(), c.d_area.as<double>(), c.d_j.p, rho, c.k0,
                     Y + ne, nt);
  SLIM_HIP(hipGetLastError());
  mark(5);
  auto out = [&](const void* src, void* dst, int64_t n) {
    if (!dst) return;
    hipLaunchKernelGGL(k_copy_out<F64>, dim3(nblk(n)), dim3(256), 0, s, src, reinterpret_cast<double2*>(dst), n);
    SLIM_HIP(hipGetLastError());
  };
  out(c.d_e.p, e_out, ne);
  out(c.d_g.p, g_out, ne);
  out(c.d_a.p, a_out, ne);
  out(c.d_phi.p, phi_out, nt);
}

}  // namespace

void launch_cast_c128_to_c64(const void* in, void* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_c128_to_c64, dim3(nblk(n)), dim3(256), 0, s, reinterpret_cast<const double2*>(in),
                     reinterpret_cast<float2*>(out), n);
  SLIM_HIP(hipGetLastError());
}
void launch_cast_c64_to_c128(const void* in, void* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_c64_to_c128, dim3(nblk(n)), dim3(256), 0, s, reinterpret_cast<const float2*>(in),
                     reinterpret_cast<double2*>(out), n);
  SLIM_HIP(hipGetLastError());
}
void launch_pack_block(const double* Z, const double* M, int n, Cplx<float>* hi, Cplx<float>* lo, hipStream_t s) {
  const int ld = (n + 1) & ~1;
  const int64_t tot = int64_t(2 * n) * ld;
  hipLaunchKernelGGL(k_pack_block, dim3(nblk(tot)), dim3(256), 0, s, reinterpret_cast<const double2*>(Z),
                     reinterpret_cast<const double2*>(M), n, ld, reinterpret_cast<float2*>(hi),
                     reinterpret_cast<float2*>(lo));
  SLIM_HIP(hipGetLastError());
}
void launch_pack_dense(const double* A, int64_t rows, int64_t cols, Cplx<float>* hi, Cplx<float>* lo, hipStream_t s) {
  const int64_t n = rows * cols;
  hipLaunchKernelGGL(k_pack_dense, dim3(nblk(n)), dim3(256), 0, s, reinterpret_cast<const double2*>(A), n,
                     reinterpret_cast<float2*>(hi), reinterpret_cast<float2*>(lo));
  SLIM_HIP(hipGetLastError());
}
void launch_add_scaled_ix(double* B, const int32_t* col, const double* val, int e0, int n, double half, hipStream_t s) {
  hipLaunchKernelGGL(k_add_ix, dim3(nblk(n)), dim3(256), 0, s, reinterpret_cast<double2*>(B), col, val, e0, n, half);
  SLIM_HIP(hipGetLastError());
}
void launch_usolve_block(const double* U, int64_t ld, int i0, int nb, double* X, int64_t ldx, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_usolve_block, dim3(nblk(nrhs)), dim3(256), 0, s, reinterpret_cast<const double2*>(U), ld, i0, nb,
                     reinterpret_cast<double2*>(X), ldx, nrhs);
  SLIM_HIP(hipGetLastError());
}
void launch_scale(double* M, int64_t n, cd f, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(256), 0, s, reinterpret_cast<double2*>(M), n, f.real(), f.imag());
  SLIM_HIP(hipGetLastError());
}

void Ctx::prof_mark(int stage, hipStream_t s) {
  std::vector<hipEvent_t>& v = prof_ev[stage];
  if (prof_used[stage] == v.size()) {
    hipEvent_t e;
    SLIM_HIP(hipEventCreate(&e));
    v.push_back(e);
  }
  SLIM_HIP(hipEventRecord(v[prof_used[stage]++], s));
}

void Ctx::drop_graphs() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  graphs.clear();
}

// The whole product captured once per (precision, x, y) on the library's stream
// and replayed on the caller's stream.  Capturing records only kernel launches.
void matvec_graph(Ctx& c, slim_prec prec, const void* x, void* y, hipStream_t s) {
  hipGraphExec_t exec = nullptr;
  for (auto& g : c.graphs)
    if (g.first.prec == int(prec) && g.first.x == x && g.first.y == y) exec = g.second;
  if (!exec) {
    hipGraph_t graph = nullptr;
    SLIM_HIP(hipStreamBeginCapture(c.s_aux, hipStreamCaptureModeThreadLocal));
    try {
      matvec(c, prec, x, y, nullptr, nullptr, nullptr, nullptr, c.s_aux);
    } catch (...) {
      (void)hipStreamEndCapture(c.s_aux, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    SLIM_HIP(hipStreamEndCapture(c.s_aux, &graph));
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    SLIM_HIP(e);
    if (c.graphs.size() >= 8) c.drop_graphs();
    c.graphs.push_back({Ctx::GraphKey{int(prec), x, y}, exec});
  }
  SLIM_HIP(hipGraphLaunch(exec, s));
}

// ms per mixed product on the library's stream, through the path slim_matvec
// takes (graph replay when graphs are on, eager launches otherwise)
double time_product(Ctx& c, int reps) {
  hipStream_t s = c.s_aux;
  const int64_t n = c.rwg.n_e + c.rwg.n_t;
  DevBuf x, y;
  x.alloc(size_t(n) * 16);
  y.alloc(size_t(n) * 16);
  SLIM_HIP(hipMemsetAsync(x.p, 0, x.bytes, s));
  hipEvent_t a, b;
  SLIM_HIP(hipEventCreate(&a));
  SLIM_HIP(hipEventCreate(&b));
  auto run = [&]() {
    if (c.opts.use_graphs) matvec_graph(c, SLIM_MIXED, x.p, y.p, s);
    else matvec(c, SLIM_MIXED, x.p, y.p, nullptr, nullptr, nullptr, nullptr, s);
  };
  run();
  SLIM_HIP(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) run();
  SLIM_HIP(hipEventRecord(b, s));
  SLIM_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  SLIM_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  c.drop_graphs();   // captured for the temporary vectors freed below
  return double(ms) / reps;
}

double time_internal(Ctx& c, int reps) {
  hipStream_t s = c.s_aux;
  hipEvent_t a, b;
  SLIM_HIP(hipEventCreate(&a));
  SLIM_HIP(hipEventCreate(&b));
  internal_launch<false>(c, c.d_x64.p, c.d_e.p, c.d_j.p, nullptr, s);
  SLIM_HIP(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) internal_launch<false>(c, c.d_x64.p, c.d_e.p, c.d_j.p, nullptr, s);
  SLIM_HIP(hipEventRecord(b, s));
  SLIM_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  SLIM_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return double(ms) / reps;
}

void matvec(Ctx& c, slim_prec prec, const void* x, void* y, void* e_out, void* g_out, void* a_out, void* phi_out,
            hipStream_t s) {
  if (prec == SLIM_FP64) matvec_t<true>(c, x, y, e_out, g_out, a_out, phi_out, s);
  else matvec_t<false>(c, x, y, e_out, g_out, a_out, phi_out, s);
}

// Internal part alone: H (complex128) -> e = Z H, g = M H (complex128 outputs).
void internal_apply(Ctx& c, slim_prec prec, const void* H, void* e, void* g, hipStream_t s, bool /*h_is_c128*/) {
  const int64_t ne = c.rwg.n_e;
  if (prec == SLIM_FP64) {
    internal_launch<true>(c, H, c.d_e.p, c.d_j.p, c.d_g.p, s);
    if (e) hipLaunchKernelGGL(k_copy_out<true>, dim3(nblk(ne)), dim3(256), 0, s, c.d_e.p, reinterpret_cast<double2*>(e), ne);
    if (g) hipLaunchKernelGGL(k_copy_out<true>, dim3(nblk(ne)), dim3(256), 0, s, c.d_g.p, reinterpret_cast<double2*>(g), ne);
  } else {
    launch_cast_c128_to_c64(H, c.d_x64.p, ne, s);
    internal_launch<false>(c, c.d_x64.p, c.d_e.p, c.d_j.p, c.d_g.p, s);
    if (e) hipLaunchKernelGGL(k_copy_out<false>, dim3(nblk(ne)), dim3(256), 0, s, c.d_e.p, reinterpret_cast<double2*>(e), ne);
    if (g) hipLaunchKernelGGL(k_copy_out<false>, dim3(nblk(ne)), dim3(256), 0, s, c.d_g.p, reinterpret_cast<double2*>(g), ne);
  }
  SLIM_HIP(hipGetLastError());
}

}  // namespace slim
