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
// rows [row0, 2n) of [Z; M]: element i of the output is row row0 + i / ld, column i % ld
__global__ void k_pack_block(const double2* Z, const double2* M, int n, int row0, int ld, float2* hi, float2* lo) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t tot = int64_t(2 * n - row0) * ld;
  if (i >= tot) return;
  const int row = row0 + int(i / ld), col = int(i % ld);
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

// Sparse Z~: the entries on the pattern (local rows / columns of a column-major n x n
// matrix), in FP64 and as complex64 hi + lo; and back into a zeroed dense copy.
__global__ void k_z_gather(const double2* Z, int n, const int32_t* rows, const int32_t* cols, int64_t nnz,
                           double2* vals, float2* hi, float2* lo) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double2 v = Z[rows[k] + int64_t(cols[k]) * n];
  vals[k] = v;
  const float2 h = make_float2(float(v.x), float(v.y));
  hi[k] = h;
  lo[k] = make_float2(float(v.x - double(h.x)), float(v.y - double(h.y)));
}
__global__ void k_z_scatter(double2* Z, int n, const int32_t* rows, const int32_t* cols, int64_t nnz,
                            const double2* vals) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  Z[rows[k] + int64_t(cols[k]) * n] = vals[k];
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

// Work list of one launch of a persistent internal kernel: static per-slot queues
// (slot s takes tiles [start[s], start[s+1])) or, when ctr is set, one dynamic queue
// tiles[first, first + count) in list order, each workgroup drawing its next tile
// from the counter when it finishes the last one.  A launch on a counter draws
// exactly count + gridDim.x tickets (every workgroup stops at its first ticket past
// the list), so the counter needs no reset between launches: ticket t stands for
// list position t mod (count + gridDim.x).  Launches on one counter must not overlap.
struct TileQueue {
  const int4* tiles;
  const int32_t* start;        // static: slot ranges (absolute tile indices) of nslots slots
  unsigned long long* ctr;     // dynamic: ticket counter (null: static)
  int32_t first, count;
  int32_t nslots;              // static: workgroups at or past nslots have no queue
};

__device__ __forceinline__ int queue_begin(const TileQueue& q) {
  return (q.ctr || int(blockIdx.x) >= q.nslots) ? 0 : q.start[blockIdx.x];
}

// Index of the workgroup's next tile, or -1 when it has none.  Every thread of the
// workgroup calls it (the dynamic form has barriers); `it` starts at
// queue_begin(q) and s_next is a workgroup-shared int.
__device__ __forceinline__ int next_tile(const TileQueue& q, int& it, int* s_next) {
  if (!q.ctr) return (int(blockIdx.x) < q.nslots && it < q.start[blockIdx.x + 1]) ? it++ : -1;
  if (threadIdx.x == 0) {
    const unsigned long long T = (unsigned long long)(q.count) + gridDim.x;
    const unsigned long long t = atomicAdd(q.ctr, 1ull) % T;
    *s_next = t < (unsigned long long)(q.count) ? q.first + int(t) : -1;
  }
  __syncthreads();
  const int ti = *s_next;
  __syncthreads();
  return ti;
}

template <bool F64, int RW>
__global__ void __launch_bounds__(256) k_internal(const float2* __restrict__ hi, const float2* __restrict__ lo,
                                                  const BlockDev* __restrict__ blocks, const TileQueue q,
                                                  const void* __restrict__ Hv, void* __restrict__ ev,
                                                  void* __restrict__ jv, void* __restrict__ gv,
                                                  unsigned long long* __restrict__ stamps,
                                                  unsigned long long* __restrict__ span) {
  using T = typename P<F64>::T;
  // RW rows per wave per sweep (chosen at the launch: 2 in FP64, where hi + lo doubles the loads; 4 or 8 in mixed)
  const C2<T>* H = reinterpret_cast<const C2<T>*>(Hv);
  C2<T>* e = reinterpret_cast<C2<T>*>(ev);
  C2<T>* jo = reinterpret_cast<C2<T>*>(jv);
  C2<T>* go = reinterpret_cast<C2<T>*>(gv);
  const int slot = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (span && threadIdx.x == 0) span[2 * slot] = wall_clock64();
  __shared__ int s_next;
  int it = queue_begin(q);
  for (int ti = next_tile(q, it, &s_next); ti >= 0; ti = next_tile(q, it, &s_next)) {
    const int4 tl = q.tiles[ti];      // block, row0, rows, slot
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
  if (span) {
    __syncthreads();
    if (threadIdx.x == 0) span[2 * slot + 1] = wall_clock64();
  }
}

// ---------------------------------------------------------------------------
// A1 + A2 for a block of right-hand sides (mixed precision) on the matrix cores.
// Every tile's rows of [Z_i; M_i] multiply up to 64 columns of H at once with
// v_mfma_f32_16x16x32_bf16.  Split-BF16: a value v (FP32, the hi part of the arena
// or the complex64 copy of H) is v_hi = bf16(v), v_lo = bf16(v - v_hi); a product
// a b is taken as a_hi b_hi + a_hi b_lo + a_lo b_hi with FP32 accumulation (the
// dropped a_lo b_lo and the split remainders are about 2^-16 of |a b|).  The complex
// product is four real ones, Re = Ar Hr - Ai Hi, Im = Ar Hi + Ai Hr: 12 MFMAs per 32
// columns of A per 16 right-hand sides.
// Operand layout of the 16x16x32 MFMA in a wave: lane l holds row (l & 15) of A and
// column (l & 15) of B, each at eight K slots; the result gives lane l column (l & 15),
// rows 4 (l >> 4) ... + 3.  The sum runs over K in any order that A and B share, so
// the slots of lane group g = l >> 4 are taken as the column pairs 8 p + 2 g, + 1
// (p = 0..3) of a 32-column chunk: in each 16-byte load the four lane groups of a row
// read 64 contiguous bytes.  The split planes of H are stored chunk by chunk, each
// chunk as [column][32 K slots] in that order: a lane's eight values are contiguous,
// and the 64 lanes of a column group read one contiguous kilobyte.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 h = __bf16(v[i]);
    hi[i] = h;
    lo[i] = __bf16(v[i] - float(h));
  }
}

// H (complex128, the first ne entries of the columns of X, leading dimension nsys)
// -> the complex64 copy H64 [R][ne] and the four split planes (re hi, re lo, im hi,
// im lo), each [chunk][column (ncol)][32].  Block i occupies whole 32-entry chunks
// (hpos maps an edge to chunk * 32 + slot, the slot in the MFMA kernel's K order), so
// that the kernel's 16-byte loads are aligned and contiguous; the entries past n_i
// stay zero from the allocation.
__global__ void k_split_h(const double2* X, int64_t nsys, int64_t ne, int R, int ncol, int64_t plane,
                          const int32_t* hpos, float2* H64, __bf16* Hs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(R) * ne) return;
  const int col = int(i / ne);
  const int64_t k = i % ne;
  const double2 v = X[int64_t(col) * nsys + k];
  const float re = float(v.x), im = float(v.y);
  H64[i] = make_float2(re, im);
  const int32_t hp = hpos[k];
  const int64_t o = (int64_t(hp >> 5) * ncol + col) * 32 + (hp & 31);
  const __bf16 rh = __bf16(re), ih = __bf16(im);
  Hs[o] = rh;
  Hs[plane + o] = __bf16(re - float(rh));
  Hs[2 * plane + o] = ih;
  Hs[3 * plane + o] = __bf16(im - float(ih));
}

// A workgroup sweeps 64 rows of a tile at a time, one 16-row group per wave, times NCG
// 16-column groups.  The four waves share each K chunk of H: its split fragments
// (4 planes x 16 NCG columns x 32 slots, contiguous in every plane) are loaded by the
// whole workgroup, one 16-byte piece per thread and column group, into one of two LDS
// buffers while the previous chunk's MFMAs run, with one barrier per chunk.  Each wave
// loads the next chunk's A fragments (HBM) the same way.  Within a column group the 12
// products are issued term by term over the four accumulators.  Every wave runs the
// same number of sweeps (rows past the tile masked), so the barriers are uniform.
template <int NCG, int RG>
__global__ void __launch_bounds__(256) k_internal_mfma(const float2* __restrict__ hi, const BlockDev* __restrict__ blocks,
                                                       const TileQueue q0, const TileQueue q1,
                                                       const int64_t* __restrict__ hoff, const __bf16* __restrict__ Hs,
                                                       int64_t plane, int ldc, int col0,
                                                       const float2* __restrict__ H64, int64_t ne, int ncol,
                                                       float2* __restrict__ E, float2* __restrict__ J) {
  static_assert(RG == 1, "one 16-row group per wave");
  constexpr int PIECES = 64 * NCG;        // 16-byte pieces of one plane's chunk (16 NCG columns x 32 slots)
  __shared__ bf16x8 hbuf[2][4 * PIECES];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  __shared__ int s_next;
  // the two phases' lists (rows of M_i, then rows of Z_i), one after the other
  for (int phase = 0; phase < 2; ++phase) {
   const TileQueue& q = phase == 0 ? q0 : q1;
   int it = queue_begin(q);
   for (int ti = next_tile(q, it, &s_next); ti >= 0; ti = next_tile(q, it, &s_next)) {
    const int4 tl = q.tiles[ti];
    const BlockDev B = blocks[tl.x];
    const int n = B.n, ld = (n + 1) & ~1, rend = tl.y + tl.z;
    const int64_t h0 = hoff[tl.x];
    // the workgroup's pieces of a chunk: piece p = threadIdx.x + 256 j -> plane p / PIECES
    auto load_h = [&](int k0, bf16x8* hs) {
      const int64_t cb = (((h0 + k0) >> 5) * ldc + col0) * 32;
#pragma unroll
      for (int j = 0; j < NCG; ++j) {
        const int p = threadIdx.x + 256 * j, pl = p / PIECES, w = p % PIECES;
        hs[j] = *reinterpret_cast<const bf16x8*>(Hs + pl * plane + cb + 8 * w);
      }
    };
    auto store_h = [&](int buf, const bf16x8* hs) {
#pragma unroll
      for (int j = 0; j < NCG; ++j) hbuf[buf][threadIdx.x + 256 * j] = hs[j];
    };
    for (int r0s = tl.y; r0s < rend; r0s += 64) {
      const int r0 = r0s + 16 * wave;
      f32x4 acc[NCG][4];
#pragma unroll
      for (int g = 0; g < NCG; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[g][q] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int row = r0 + lr;
      const float2* arow = hi + (B.off + int64_t(row) * ld);
      // A fragment of the K chunk at k0: 8 complex (4 pairs), zero past the tile or row
      auto load_a = [&](int k0, float4* a) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int kk = k0 + 8 * p + 2 * lg;
          a[p] = (row < rend && kk < ld) ? ntload(arow + kk) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      };
      float4 a_cur[4], a_nxt[4];
      bf16x8 hs[NCG];
      load_h(0, hs);
      load_a(0, a_cur);
      store_h(0, hs);
      __syncthreads();
      int buf = 0;
      for (int k0 = 0; k0 < n; k0 += 32) {
        const bool more = k0 + 32 < n;
        if (more) {
          load_a(k0 + 32, a_nxt);
          load_h(k0 + 32, hs);
        }
        bf16x8 ah[2], al[2];   // [0]: real part, [1]: imaginary part
        {
          float re[8], im[8];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            re[2 * p] = a_cur[p].x; im[2 * p] = a_cur[p].y;
            re[2 * p + 1] = a_cur[p].z; im[2 * p + 1] = a_cur[p].w;
          }
          split_bf16(re, ah[0], al[0]);
          split_bf16(im, ah[1], al[1]);
        }
        // accumulators: 0 = Ar Hr, 1 = Ai Hi, 2 = Ar Hi, 3 = Ai Hr; planes: 0 Hr hi, 1 Hr lo, 2 Hi hi, 3 Hi lo
        // term 0: a_hi b_hi, term 1: a_hi b_lo, term 2: a_lo b_hi
#pragma unroll
        for (int g = 0; g < NCG; ++g) {
          bf16x8 hv[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) hv[pl] = hbuf[buf][pl * PIECES + (16 * g + lr) * 4 + lg];
#pragma unroll
          for (int term = 0; term < 3; ++term)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int ai = (q == 0 || q == 2) ? 0 : 1;     // Ar for accumulators 0, 2; Ai for 1, 3
              const int bp = (q == 0 || q == 3) ? 0 : 2;     // Hr for accumulators 0, 3; Hi for 1, 2
              const bf16x8 av = term == 2 ? al[ai] : ah[ai];
              const bf16x8 bv = term == 1 ? hv[bp + 1] : hv[bp];
              acc[g][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[g][q], 0, 0, 0);
            }
        }
        if (more) {
          store_h(buf ^ 1, hs);
#pragma unroll
          for (int p = 0; p < 4; ++p) a_cur[p] = a_nxt[p];
        }
        __syncthreads();   // the next chunk is in LDS; this one may be overwritten
        buf ^= 1;
      }
      // epilogue: e rows (row < n) and j = H - g rows (row >= n), column 16 g + lr
#pragma unroll
      for (int g = 0; g < NCG; ++g) {
        const int col = 16 * g + lr;
        if (col >= ncol) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = r0 + 4 * lg + q;
          if (rr >= rend) continue;
          const float yr = acc[g][0][q] - acc[g][1][q], yi = acc[g][2][q] + acc[g][3][q];
          if (rr < n) {
            E[int64_t(col) * ne + B.e0 + rr] = make_float2(yr, yi);
          } else {
            const int64_t k = int64_t(col) * ne + B.e0 + (rr - n);
            const float2 h = H64[k];
            J[k] = make_float2(h.x - yr, h.y - yi);
          }
        }
      }
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
// Sum over the LPR lanes of a row group (LPR a power of two up to 64).
template <int LPR, bool F64>
__device__ __forceinline__ typename P<F64>::T row_sum(typename P<F64>::T v) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
  return v;
}

// A5 + A6 for pulses: phi_t = W_rho Phi_rho + L_phi,NR (B c0rho); sixteen lanes per row
// (four rows per wave), two entries per lane per trip.
template <bool F64>
__global__ void __launch_bounds__(256) k_phi(const int32_t* wt_base, const void* wt_w, const void* octv, int64_t N3,
                                             int Nx, int NxNy, const int64_t* ptr, const int32_t* col,
                                             const void* valv, const void* rhov, void* phiv, int64_t n_t) {
  using T = typename P<F64>::T;
  constexpr int LPR = 16;
  const int64_t t = (int64_t(blockIdx.x) * 256 + threadIdx.x) / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  const bool live = t < n_t;      // every lane stays for the shuffles
  T sr = 0, si = 0;
  if (live) {
    const T* w = reinterpret_cast<const T*>(wt_w);
    const C2<T>* Phi = reinterpret_cast<const C2<T>*>(octv) + 3 * N3;
    const C2<T>* val = reinterpret_cast<const C2<T>*>(valv);
    const C2<T>* rho = reinterpret_cast<const C2<T>*>(rhov);
    const int64_t base = wt_base[t];
#pragma unroll
    for (int k = lane; k < 27; k += LPR) {
      const int64_t node = base + (k % 3) + Nx * ((k / 3) % 3) + int64_t(NxNy) * (k / 9);
      const T wv = w[27 * t + k];
      sr += wv * Phi[node].x;
      si += wv * Phi[node].y;
    }
    const int64_t zend = ptr[t + 1];
    for (int64_t z = ptr[t] + lane; z < zend; z += 2 * LPR) {
      const bool two = z + LPR < zend;
      const int c0 = col[z], c1 = two ? col[z + LPR] : c0;
      const C2<T> a0 = val[z], a1 = two ? val[z + LPR] : C2<T>{T(0), T(0)};
      const C2<T> b0 = rho[c0], b1 = rho[c1];
      sr += a0.x * b0.x - a0.y * b0.y + a1.x * b1.x - a1.y * b1.y;
      si += a0.x * b0.y + a0.y * b0.x + a1.x * b1.y + a1.y * b1.x;
    }
  }
  sr = row_sum<LPR, F64>(sr);
  si = row_sum<LPR, F64>(si);
  if (live && lane == 0) reinterpret_cast<C2<T>*>(phiv)[t] = {sr, si};
}

// ---------------------------------------------------------------------------
// A5 + A6 + A7 for RWG rows: a = W_A Phi + L_A,NR j;
// y1 = j k0 a + l (phi[T+] - phi[T-]) + I_x e / eta0  (written as complex128).
// ---------------------------------------------------------------------------
// Sixteen lanes per RWG row (four rows per wave): the 27-node W gather takes two
// passes, the near-field row (about 265 entries at the 2000-conductor workload) is
// strided two entries per lane per trip, and the row tail (phi of T+-, the I_x
// entries) runs on the first lane of each row group, four rows at a time per wave.
template <bool F64, bool AIM>
__global__ void __launch_bounds__(256) k_rows_A(const int32_t* we_base, const void* we_w, const void* octv, int64_t N3,
                                                int Nx, int NxNy, const int64_t* ptr, const int32_t* col,
                                                const void* valv, const void* jv, const void* a_dense,
                                                const void* phiv, const void* ev, const int32_t* tplus,
                                                const int32_t* tminus, const double* len, const int32_t* ix_col,
                                                const double* ix_val, double k0, double inv_eta0, void* av,
                                                double2* y, int64_t n_e) {
  using T = typename P<F64>::T;
  constexpr int LPR = 16;
  const int64_t m = (int64_t(blockIdx.x) * 256 + threadIdx.x) / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  const bool live = m < n_e;      // every lane stays for the shuffles
  T sr = 0, si = 0;
  if (AIM) {
    if (live) {
      const T* w = reinterpret_cast<const T*>(we_w) + 81 * m;
      const C2<T>* Phi = reinterpret_cast<const C2<T>*>(octv);
      const int64_t base = we_base[m];
#pragma unroll
      for (int k = lane; k < 27; k += LPR) {
        const int64_t node = base + (k % 3) + Nx * ((k / 3) % 3) + int64_t(NxNy) * (k / 9);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C2<T> p = Phi[c * N3 + node];
          sr += w[c * 27 + k] * p.x;
          si += w[c * 27 + k] * p.y;
        }
      }
      const C2<T>* val = reinterpret_cast<const C2<T>*>(valv);
      const C2<T>* j = reinterpret_cast<const C2<T>*>(jv);
      // two entries per lane per trip: both column loads, then both gathers, are in flight together
      const int64_t zend = ptr[m + 1];
      for (int64_t z = ptr[m] + lane; z < zend; z += 2 * LPR) {
        const bool two = z + LPR < zend;
        const int c0 = col[z], c1 = two ? col[z + LPR] : c0;
        const C2<T> a0 = val[z], a1 = two ? val[z + LPR] : C2<T>{T(0), T(0)};
        const C2<T> b0 = j[c0], b1 = j[c1];
        sr += a0.x * b0.x - a0.y * b0.y + a1.x * b1.x - a1.y * b1.y;
        si += a0.x * b0.y + a0.y * b0.x + a1.x * b1.y + a1.y * b1.x;
      }
    }
    sr = row_sum<LPR, F64>(sr);
    si = row_sum<LPR, F64>(si);
  } else if (live && lane == 0) {
    const C2<T> a = reinterpret_cast<const C2<T>*>(a_dense)[m];
    sr = a.x;
    si = a.y;
  }
  if (live && lane == 0) {
    const C2<T>* phi = reinterpret_cast<const C2<T>*>(phiv);
    const C2<T>* e = reinterpret_cast<const C2<T>*>(ev);
    if (AIM) reinterpret_cast<C2<T>*>(av)[m] = {sr, si};
    const double l = len[m];
    const C2<T> pp = phi[tplus[m]], pm = phi[tminus[m]];
    double yr = -k0 * double(si) + l * (double(pp.x) - double(pm.x));
    double yi = k0 * double(sr) + l * (double(pp.y) - double(pm.y));
    // without e (ev null) the I_x e / eta0 term is left to k_add_ix_e, which adds it in
    // the same order, so the result is the same to the bit
    for (int q = 0; e && q < 4; ++q) {
      const int c = ix_col[4 * m + q];
      if (c < 0) continue;
      const C2<T> ec = e[c];
      yr += inv_eta0 * ix_val[4 * m + q] * double(ec.x);
      yi += inv_eta0 * ix_val[4 * m + q] * double(ec.y);
    }
    y[m] = make_double2(yr, yi);
  }
}

// y1 += I_x e / eta0: the last term of the RWG rows, once the rows of Z_i are done
template <bool F64>
__global__ void k_add_ix_e(const int32_t* __restrict__ ix_col, const double* __restrict__ ix_val, const void* ev,
                           double inv_eta0, double2* __restrict__ y, int64_t n_e) {
  using T = typename P<F64>::T;
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= n_e) return;
  const C2<T>* e = reinterpret_cast<const C2<T>*>(ev);
  double2 v = y[m];
  for (int q = 0; q < 4; ++q) {
    const int c = ix_col[4 * m + q];
    if (c < 0) continue;
    const C2<T> ec = e[c];
    v.x += inv_eta0 * ix_val[4 * m + q] * double(ec.x);
    v.y += inv_eta0 * ix_val[4 * m + q] * double(ec.y);
  }
  y[m] = v;
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

// e = Z~ H with the sparse Z~ of the high-frequency form (CSR over all RWG rows, global
// columns, complex64 hi + lo values; FP64 adds lo).  Eight lanes per row stride its
// entries; the partial sums meet through lane shuffles.
template <bool F64>
__global__ void __launch_bounds__(256) k_zsparse(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                 const float2* __restrict__ vhi, const float2* __restrict__ vlo,
                                                 const void* __restrict__ Hv, void* __restrict__ ev, int64_t n) {
  using T = typename P<F64>::T;
  const C2<T>* H = reinterpret_cast<const C2<T>*>(Hv);
  C2<T>* e = reinterpret_cast<C2<T>*>(ev);
  const int64_t row = (int64_t(blockIdx.x) * 256 + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  T sr = 0, si = 0;
  if (row < n) {
    for (int64_t k = ptr[row] + sub; k < ptr[row + 1]; k += 8) {
      const C2<T> h = H[col[k]];
      const float2 a = vhi[k];
      T ar = a.x, ai = a.y;
      if (F64) {
        const float2 b = vlo[k];
        ar += T(b.x);
        ai += T(b.y);
      }
      sr += ar * h.x - ai * h.y;
      si += ar * h.y + ai * h.x;
    }
  }
  sr = group_sum8<F64>(sr);
  si = group_sum8<F64>(si);
  if (sub == 0 && row < n) e[row] = {sr, si};
}

// Work list of a phase of the internal tiles (0: rows of M_i, 1: rows of Z_i) on
// dynamic-dispatch counter `ctr` (used in the dynamic scheduling modes).
TileQueue phase_queue(Ctx& c, int phase, int ctr) {
  TileQueue q;
  q.tiles = c.d_tiles.as<int4>();
  q.start = c.d_slot_start.as<int32_t>() + (phase == 0 ? 0 : size_t(c.slots + 1));
  q.ctr = c.dynamic ? c.d_qctr.as<unsigned long long>() + ctr : nullptr;
  q.first = c.phase_first[phase];
  q.count = c.phase_count[phase];
  q.nslots = phase == 0 ? c.slots : c.zslots();
  return q;
}

// One phase of the internal product: 0 = rows of M_i (g = M H, j = H - g), 1 = rows
// of Z_i (e = Z H); phase -1 runs both, one after the other, on stream s.
template <bool F64>
void internal_launch(Ctx& c, const void* H, void* e, void* j, void* g, hipStream_t s, int phase = -1) {
  if (phase < 0) {
    internal_launch<F64>(c, H, e, j, g, s, 0);
    internal_launch<F64>(c, H, e, j, g, s, 1);
    return;
  }
  if (phase == 1 && c.hf_sparse) {
    // rows of Z~: the sparse product of the high-frequency form
    const int64_t ne = c.rwg.n_e;
    hipLaunchKernelGGL(k_zsparse<F64>, dim3(nblk(8 * ne)), dim3(256), 0, s, c.d_zs_ptr.as<int64_t>(),
                       c.d_zs_col.as<int32_t>(), c.d_zs_hi.as<float2>(), c.d_zs_lo.as<float2>(), H, e, ne);
    SLIM_HIP(hipGetLastError());
    return;
  }
  unsigned long long* st = c.record ? c.d_stamps.as<unsigned long long>() : nullptr;
  unsigned long long* sp = c.gprof_on ? c.d_span.as<unsigned long long>() + 2 * size_t(phase == 0 ? 0 : c.slots) : nullptr;
  // the FP64 rows of Z_i on a grid of their own take a counter of their own
  const bool own = phase == 1 && c.zgrid(F64) != c.zslots();
  const TileQueue q = phase_queue(c, phase, own ? 4 : phase);
  const unsigned nwg = unsigned(phase == 0 ? c.slots : c.zgrid(F64));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), 0, s, c.d_hi.as<float2>(), c.d_lo.as<float2>(),
                       c.d_blocks.as<BlockDev>(), q, H, e, j, g, st, sp);
  };
  if (F64) go(k_internal<true, 2>);   // two rows per wave: 120 VGPRs, four waves per SIMD
  else if (c.rw_mixed == 4) go(k_internal<false, 4>);
  else go(k_internal<false, 8>);
  SLIM_HIP(hipGetLastError());
}

// ext_e, ext_j: the internal part's e = Z H and j = H - M H (precision of the path)
// computed elsewhere; the product then runs only its external part on them.
template <bool F64>
void matvec_t(Ctx& c, const void* x, void* y, void* e_out, void* g_out, void* a_out, void* phi_out, hipStream_t s,
              void* ext_e = nullptr, void* ext_j = nullptr) {
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
    hipLaunchKernelGGL(k_phi<F64>, dim3(nblk(nt, 16)), dim3(256), 0, st, c.d_wt_base.as<int32_t>(),
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
  void* ev = ext_e ? ext_e : c.d_e.p;
  void* jv = ext_j ? ext_j : c.d_j.p;
  // The rows of Z_i (e, needed only by the RWG rows at the end) run on a third
  // stream, concurrently with the projection and the convolution of j, once the
  // rows of M_i (g, j) are done.
  const bool overlap_z = overlap && c.s_int && !ext_e;
  if (!ext_e) {
    mark(0);
    internal_launch<F64>(c, X, ev, jv, g_out ? c.d_g.p : nullptr, s, overlap_z ? 0 : -1);
    if (overlap_z) {
      SLIM_HIP(hipEventRecord(c.ev_zfork, s));
      SLIM_HIP(hipStreamWaitEvent(c.s_int, c.ev_zfork, 0));
      internal_launch<F64>(c, X, ev, jv, nullptr, c.s_int, 1);
      SLIM_HIP(hipEventRecord(c.ev_zjoin, c.s_int));
    }
    mark(0);
  }
  if (c.plain) {
    hipLaunchKernelGGL(k_dense_gemv<F64>, dim3(nblk(nt, 4)), dim3(256), 0, s, c.d_Lphi_hi.as<float2>(),
                       c.d_Lphi_lo.as<float2>(), nt, rho, c.d_area.as<double>(), c.d_phi.p);
    hipLaunchKernelGGL(k_dense_gemv<F64>, dim3(nblk(ne, 4)), dim3(256), 0, s, c.d_LA_hi.as<float2>(),
                       c.d_LA_lo.as<float2>(), ne, jv, nullptr, c.d_a.p);
    SLIM_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_rows_A<F64, false>), dim3(nblk(ne, 16)), dim3(256), 0, s, nullptr, nullptr, nullptr,
                       int64_t(0), 0, 0, nullptr, nullptr, nullptr, nullptr, c.d_a.p, c.d_phi.p, ev,
                       c.d_tplus.as<int32_t>(), c.d_tminus.as<int32_t>(), c.d_len.as<double>(),
                       c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), c.k0, inv_eta0, nullptr, Y, ne);
  } else {
    mark(1);
    hipLaunchKernelGGL(k_project<F64>, dim3(nblk(8 * (c.n_pe_nodes + (overlap ? 0 : c.n_pt_nodes)))), dim3(256), 0, s,
                       c.d_pe_node.as<int32_t>(), c.d_pe_ptr.as<int32_t>(), c.d_pe_idx.as<int32_t>(),
                       F64 ? c.d_pe_w64.p : c.d_pe_w32.p, c.n_pe_nodes, c.d_pt_node.as<int32_t>(),
                       c.d_pt_ptr.as<int32_t>(), c.d_pt_idx.as<int32_t>(), F64 ? c.d_pt_w64.p : c.d_pt_w32.p,
                       overlap ? int64_t(0) : c.n_pt_nodes, jv, rho, oct_in, N3);
    SLIM_HIP(hipGetLastError());
    mark(1);
    mark(2);
    aim_convolve(c, F64, overlap ? 3 : 4, s, 0, c.layered);
    mark(2);
    mark(3);
    if (overlap) {
      SLIM_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
    } else {
      hipLaunchKernelGGL(k_phi<F64>, dim3(nblk(nt, 16)), dim3(256), 0, s, c.d_wt_base.as<int32_t>(),
                         F64 ? c.d_wt_w64.p : c.d_wt_w32.p, c.d_oct_out.p, N3, Nx, NxNy, c.d_nP_ptr.as<int64_t>(),
                         c.d_nP_col.as<int32_t>(), F64 ? c.d_nP_v128.p : c.d_nP_v64.p, rho, c.d_phi.p, nt);
      SLIM_HIP(hipGetLastError());
    }
    mark(3);
    mark(4);
    // with the rows of Z_i still running beside, the RWG rows take everything but the
    // I_x e / eta0 term now (their near-field and interpolation reads overlap the tail of
    // that launch) and the term is added once e is complete
    hipLaunchKernelGGL((k_rows_A<F64, true>), dim3(nblk(ne, 16)), dim3(256), 0, s, c.d_we_base.as<int32_t>(),
                       F64 ? c.d_we_w64.p : c.d_we_w32.p, c.d_oct_out.p, N3, Nx, NxNy, c.d_nA_ptr.as<int64_t>(),
                       c.d_nA_col.as<int32_t>(), F64 ? c.d_nA_v128.p : c.d_nA_v64.p, jv, nullptr, c.d_phi.p,
                       overlap_z ? nullptr : ev, c.d_tplus.as<int32_t>(), c.d_tminus.as<int32_t>(),
                       c.d_len.as<double>(), c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), c.k0, inv_eta0,
                       c.d_a.p, Y, ne);
    mark(4);
  }
  SLIM_HIP(hipGetLastError());
  mark(5);
  hipLaunchKernelGGL(k_rows_T<F64>, dim3(nblk(nt)), dim3(256), 0, s, c.d_tri_edge.as<int32_t>(),
                     c.d_tri_sign.as<int8_t>(), c.d_len.as<double>(), c.d_area.as<double>(), jv, rho, c.k0,
                     Y + ne, nt);
  SLIM_HIP(hipGetLastError());
  mark(5);
  if (overlap_z) {
    SLIM_HIP(hipStreamWaitEvent(s, c.ev_zjoin, 0));
    hipLaunchKernelGGL(k_add_ix_e<F64>, dim3(nblk(ne)), dim3(256), 0, s, c.d_ix_col.as<int32_t>(),
                       c.d_ix_val.as<double>(), ev, inv_eta0, Y, ne);
    SLIM_HIP(hipGetLastError());
  }
  auto out = [&](const void* src, void* dst, int64_t n) {
    if (!dst) return;
    hipLaunchKernelGGL(k_copy_out<F64>, dim3(nblk(n)), dim3(256), 0, s, src, reinterpret_cast<double2*>(dst), n);
    SLIM_HIP(hipGetLastError());
  };
  out(ev, e_out, ne);
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
void launch_pack_block(const double* Z, const double* M, int n, int row0, Cplx<float>* hi, Cplx<float>* lo,
                       hipStream_t s) {
  const int ld = (n + 1) & ~1;
  const int64_t tot = int64_t(2 * n - row0) * ld;
  hipLaunchKernelGGL(k_pack_block, dim3(nblk(tot)), dim3(256), 0, s, reinterpret_cast<const double2*>(Z),
                     reinterpret_cast<const double2*>(M), n, row0, ld, reinterpret_cast<float2*>(hi),
                     reinterpret_cast<float2*>(lo));
  SLIM_HIP(hipGetLastError());
}
void launch_z_gather_mask(double* Z, int n, const int32_t* rows, const int32_t* cols, int64_t nnz, double* vals,
                          Cplx<float>* hi, Cplx<float>* lo, hipStream_t s) {
  if (nnz > 0) {
    hipLaunchKernelGGL(k_z_gather, dim3(nblk(nnz)), dim3(256), 0, s, reinterpret_cast<const double2*>(Z), n, rows, cols,
                       nnz, reinterpret_cast<double2*>(vals), reinterpret_cast<float2*>(hi), reinterpret_cast<float2*>(lo));
    SLIM_HIP(hipGetLastError());
  }
  SLIM_HIP(hipMemsetAsync(Z, 0, size_t(n) * n * 16, s));
  if (nnz > 0) {
    hipLaunchKernelGGL(k_z_scatter, dim3(nblk(nnz)), dim3(256), 0, s, reinterpret_cast<double2*>(Z), n, rows, cols, nnz,
                       reinterpret_cast<const double2*>(vals));
    SLIM_HIP(hipGetLastError());
  }
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
  if (!c.gprof_on) {
    SLIM_HIP(hipGraphLaunch(exec, s));
    return;
  }
  // graph-path timing: the replay between two events on the caller's stream; the
  // internal kernel from its own wall-clock stamps (first workgroup start to last
  // workgroup end), which the captured launch writes; synchronous
  SLIM_HIP(hipEventRecord(c.gev[0], s));
  SLIM_HIP(hipGraphLaunch(exec, s));
  SLIM_HIP(hipEventRecord(c.gev[1], s));
  SLIM_HIP(hipEventSynchronize(c.gev[1]));
  float t_all = 0.f;
  SLIM_HIP(hipEventElapsedTime(&t_all, c.gev[0], c.gev[1]));
  const int zg = c.zgrid(prec == SLIM_FP64);
  std::vector<unsigned long long> st(2 * size_t(c.slots + zg));
  SLIM_HIP(hipMemcpy(st.data(), c.d_span.p, st.size() * 8, hipMemcpyDeviceToHost));
  if (c.wall_khz <= 0) {
    int khz = 0;
    SLIM_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c.device));
    c.wall_khz = khz;
  }
  // per phase: first workgroup start to last workgroup end
  unsigned long long a0 = ~0ull, a1 = 0;
  for (int ph = 0; ph < 2; ++ph) {
    if (c.phase_count[ph] == 0) continue;   // no persistent launch (the sparse Z~ rows)
    unsigned long long t0 = ~0ull, t1 = 0;
    const size_t base = ph == 0 ? 0 : size_t(c.slots);
    for (int k = 0; k < (ph == 0 ? c.slots : zg); ++k) {
      t0 = std::min(t0, st[2 * (base + k)]);
      t1 = std::max(t1, st[2 * (base + k) + 1]);
    }
    c.gprof_ms[2 + ph] += t1 > t0 && c.wall_khz > 0 ? double(t1 - t0) / double(c.wall_khz) : 0.0;
    a0 = std::min(a0, t0);
    a1 = std::max(a1, t1);
  }
  c.gprof_ms[0] += a1 > a0 && c.wall_khz > 0 ? double(a1 - a0) / double(c.wall_khz) : 0.0;
  c.gprof_ms[1] += t_all;
  c.gprof_calls++;
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

// Y = A X for n_rhs columns.  MIXED: one split-BF16 MFMA launch of the internal blocks
// per 64 columns, then the external part column by column on the columns' e and j.
// FP64: every column through the single-column FP64 path (eager).
void matvec_block(Ctx& c, slim_prec prec, const void* X, void* Y, int R, hipStream_t s) {
  const int64_t ne = c.rwg.n_e, nsys = c.rwg.n_e + c.rwg.n_t;
  const char* Xc = reinterpret_cast<const char*>(X);
  char* Yc = reinterpret_cast<char*>(Y);
  if (prec == SLIM_FP64) {
    for (int col = 0; col < R; ++col)
      matvec_t<true>(c, Xc + size_t(col) * nsys * 16, Yc + size_t(col) * nsys * 16, nullptr, nullptr, nullptr, nullptr, s);
    return;
  }
  const int Rpad = (R + 15) & ~15;
  if (c.blk_ldh == 0) {
    // block i occupies round_up(n_i, 32) / 32 chunks of the planes; local index k sits
    // in chunk k / 32 at the slot of its K position (column pair 8 p + 2 g + e ->
    // slot 8 g + 2 p + e); hpos = chunk * 32 + slot
    std::vector<int64_t> hoff(c.blocks.size());
    std::vector<int32_t> hpos(ne);
    int64_t o = 0;
    for (size_t i = 0; i < c.blocks.size(); ++i) {
      hoff[i] = o;
      for (int k = 0; k < c.blocks[i].n; ++k) {
        const int kk = k & 31, p = kk >> 3, g = (kk >> 1) & 3, e = kk & 1;
        hpos[c.blocks[i].e0 + k] = int32_t(o + (k & ~31) + 8 * g + 2 * p + e);
      }
      o += (c.blocks[i].n + 31) & ~31;
    }
    SLIM_REQUIRE(o < (int64_t(1) << 31), SLIM_E_UNSUPPORTED, "too many unknowns for the block product");
    c.d_blk_hoff.upload(hoff);
    c.d_blk_hpos.upload(hpos);
    c.blk_ldh = o;
  }
  if (c.blk_cols < Rpad) {
    c.d_blk_hs.alloc(size_t(4) * Rpad * c.blk_ldh * 2);
    SLIM_HIP(hipMemsetAsync(c.d_blk_hs.p, 0, c.d_blk_hs.bytes, s));
    c.d_blk_h64.alloc(size_t(Rpad) * ne * 8);
    c.d_blk_e.alloc(size_t(Rpad) * ne * 8);
    c.d_blk_j.alloc(size_t(Rpad) * ne * 8);
    c.blk_cols = Rpad;
  }
  const int64_t plane = int64_t(c.blk_cols) * c.blk_ldh;
  __bf16* Hs = c.d_blk_hs.as<__bf16>();
  hipLaunchKernelGGL(k_split_h, dim3(nblk(int64_t(R) * ne)), dim3(256), 0, s, reinterpret_cast<const double2*>(X), nsys,
                     ne, R, c.blk_cols, plane, c.d_blk_hpos.as<int32_t>(), c.d_blk_h64.as<float2>(), Hs);
  SLIM_HIP(hipGetLastError());
  if (c.prof_on) c.prof_mark(0, s);
  for (int col0 = 0; col0 < R; col0 += 64) {
    const int ncol = std::min(64, R - col0), ncg = (ncol + 15) / 16;
    auto go = [&](auto kern) {
      // every static queue of both phases has its workgroup (the phases may differ in count)
      hipLaunchKernelGGL(kern, dim3(unsigned(std::max(c.slots, c.zslots()))), dim3(256), 0, s, c.d_hi.as<float2>(),
                         c.d_blocks.as<BlockDev>(),
                         phase_queue(c, 0, 2), phase_queue(c, 1, 3), c.d_blk_hoff.as<int64_t>(),
                         Hs, plane, c.blk_cols, col0, c.d_blk_h64.as<float2>() + int64_t(col0) * ne,
                         ne, ncol, c.d_blk_e.as<float2>() + int64_t(col0) * ne, c.d_blk_j.as<float2>() + int64_t(col0) * ne);
    };
    if (ncg == 1) go(k_internal_mfma<1, 1>);
    else if (ncg == 2) go(k_internal_mfma<2, 1>);
    else if (ncg == 3) go(k_internal_mfma<3, 1>);
    else go(k_internal_mfma<4, 1>);
    SLIM_HIP(hipGetLastError());
  }
  if (c.hf_sparse)   // the rows of Z~ column by column (sparse, not on the matrix cores)
    for (int col = 0; col < R; ++col) {
      hipLaunchKernelGGL(k_zsparse<false>, dim3(nblk(8 * ne)), dim3(256), 0, s, c.d_zs_ptr.as<int64_t>(),
                         c.d_zs_col.as<int32_t>(), c.d_zs_hi.as<float2>(), c.d_zs_lo.as<float2>(),
                         c.d_blk_h64.as<float2>() + int64_t(col) * ne, c.d_blk_e.as<float2>() + int64_t(col) * ne, ne);
      SLIM_HIP(hipGetLastError());
    }
  if (c.prof_on) c.prof_mark(0, s);
  for (int col = 0; col < R; ++col)
    matvec_t<false>(c, Xc + size_t(col) * nsys * 16, Yc + size_t(col) * nsys * 16, nullptr, nullptr, nullptr, nullptr, s,
                    c.d_blk_e.as<float2>() + int64_t(col) * ne, c.d_blk_j.as<float2>() + int64_t(col) * ne);
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
