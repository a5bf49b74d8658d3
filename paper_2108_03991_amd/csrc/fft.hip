// Grid convolution H of eq. (11) by FFT on the zero-padded (2N)^3 grid.
//
// One pass transforms every line along one axis.  A workgroup stages a batch of
// lines in LDS (4096 or 8192 complex64, 4096 complex128 elements), runs a Stockham
// autosort FFT with radix-8/4/2 butterflies held in registers, and writes the
// result back.  Passes of the convolution, per component (x, y, z, rho):
//   x-fwd  (reads the N^3 octant, the upper half of each line is zero)
//   y-fwd  (upper half zero)
//   z      (upper half zero; forward, times the spectrum G^, inverse; only the
//           lower half of the result is kept)
//   y-inv  (keeps the lower half)   x-inv (keeps the lower half -> octant)
// so 26 N^3 elements move per component instead of the 48 N^3 of unpruned
// passes with a separate spectrum multiply.
#include "ctx.hpp"

namespace slim {

namespace {

template <class T> struct C2 { T x, y; };
template <class T> __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward) or +i (inverse)
template <class T, bool INV> __device__ __forceinline__ C2<T> rot90(C2<T> a) {
  return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}

template <class T, bool INV> __device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <class T, bool INV> __device__ __forceinline__ void dft4(C2<T>* v) {
  C2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  C2<T> t2 = cadd(v[1], v[3]), t3 = rot90<T, INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <class T, bool INV> __device__ __forceinline__ void dft8(C2<T>* v) {
  C2<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T r = T(0.70710678118654752440);
  // w8^k for k = 0..3, w8 = e^{-i pi/4} (forward) or e^{+i pi/4} (inverse)
  C2<T> w1 = INV ? C2<T>{r, r} : C2<T>{r, -r};
  C2<T> w3 = INV ? C2<T>{-r, r} : C2<T>{-r, -r};
  C2<T> o1 = cmul(o[1], w1), o2 = rot90<T, INV>(o[2]), o3 = cmul(o[3], w3);
  v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
}

template <int R, class T, bool INV> __device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft2<T, INV>(v);
}

// One Stockham stage of radix R on every line of the LDS batch (in place through registers).
// Element j + r L/R of the input feeds output (j/Ns) Ns R + j%Ns + r Ns, after the
// twiddle e^{-+2 pi i (j%Ns) r / (Ns R)} and an R-point DFT.
constexpr int kFftThreads = 512;

// LDS layout of a batch: line b, element i at b * LP + i + i/8 with the odd
// line stride LP = L + L/8 + 1.  The padding element every eight breaks the
// 64-byte lane stride of the radix-8 write phase; the odd line stride spreads
// the lanes of the strided passes (consecutive lanes = consecutive lines) over
// all banks instead of one.
template <int L> constexpr int line_stride() { return L + L / 8 + 1; }
template <int L> __device__ __forceinline__ int pidx(int b, int i) { return b * line_stride<L>() + i + (i >> 3); }

// HIN: the upper half of each line is zero and only the lower half is read (a first
// stage, Ns = 1: input r of a butterfly is at j + r L/R, in the upper half for r >= R/2);
// HOUT: only the lower half of the result is written (a last stage, Ns = L/R: output r
// goes to k + r Ns).
template <class T, int L, int R, int ELEMS, bool INV, bool HIN = false, bool HOUT = false>
__device__ __forceinline__ void stage(C2<T>* lds, int Ns, const C2<T>* tw) {   // tw: the L twiddles
  constexpr int NB = ELEMS / R;           // butterflies in the batch
  constexpr int PER = NB / kFftThreads;   // per thread
  static_assert(NB % kFftThreads == 0, "batch too small");
  C2<T> v[PER][R];
  int outb[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int it = threadIdx.x + p * kFftThreads;
    const int line = it / (L / R), j = it % (L / R);
    const int k = j % Ns;
#pragma unroll
    for (int r = 0; r < R; ++r)
      v[p][r] = (HIN && r >= R / 2) ? C2<T>{T(0), T(0)} : lds[pidx<L>(line, j + r * (L / R))];
    if (Ns > 1) {
      // twiddles w^r, w = e^{-+2 pi i k / (Ns R)} = table entry k L/(Ns R): one table
      // read, the powers by products (depth log2 R), in place of R - 1 reads
      C2<T> w[R];
      w[1] = tw[k * (L / (Ns * R))];
      if (INV) w[1].y = -w[1].y;
      if (R >= 4) {
        w[2] = cmul(w[1], w[1]);
        w[3] = cmul(w[2], w[1]);
      }
      if (R == 8) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[p][r] = cmul(v[p][r], w[r]);
    }
    dftR<R, T, INV>(v[p]);
    outb[p] = (line << 16) | ((j / Ns) * Ns * R + k);
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (!HOUT || r < R / 2) lds[pidx<L>(outb[p] >> 16, (outb[p] & 0xffff) + r * Ns)] = v[p][r];
  __syncthreads();
}

// The stages of a batch: radix 8 while at least 8 points remain per sub-transform, then
// one of radix 4 or 2.  HIN (zero-padded input: the upper half of every line is zero)
// prunes the first stage, HOUT (only the lower half of the result is kept) the last.
template <class T, int L, int ELEMS, bool INV, bool HIN = false, bool HOUT = false, int NS = 1>
__device__ __forceinline__ void fft_batch(C2<T>* lds, const C2<T>* tw) {
  constexpr int REM = L / NS;
  constexpr int R = REM >= 8 ? 8 : REM;
  stage<T, L, R, ELEMS, INV, HIN && NS == 1, HOUT && NS * R == L>(lds, NS, tw);
  if constexpr (NS * R < L) fft_batch<T, L, ELEMS, INV, HIN, HOUT, NS * R>(lds, tw);
}

// Offset of index i along an axis of stride lo; a blocked axis (sh > 0) splits i into
// (i >> sh, i & (2^sh - 1)) with strides (hi, lo).
__device__ __forceinline__ int64_t boff(int i, int64_t lo, int64_t hi, int sh) {
  return sh ? int64_t(i >> sh) * hi + int64_t(i & ((1 << sh) - 1)) * lo : int64_t(i) * lo;
}

struct PassArgs {
  const void* in; void* out;
  int64_t in_e, in_o1, in_o2, out_e, out_o1, out_o2;
  // blocked element (e) and outer (o2) axes of the z-block layout: strides of the block index
  int64_t in_e_hi, in_o2_hi, out_e_hi, out_o2_hi;
  int in_e_sh, in_o2_sh, out_e_sh, out_o2_sh;
  int n1, n2;            // line counts along the two outer indices
  int n_in, n_out;       // elements read (others zero) / written per line
  const void* tw;        // L twiddles e^{-2 pi i m / L}
  const void* mul;       // spectrum octant for the fused pass: index k of a line of length 2h is
  int64_t mul_e, mul_o1, mul_o2;   // read at min(k, 2h - k) (the spectrum is even)
  int h_e, h_o1, h_o2;
  int64_t comp_in, comp_out;   // component strides (blockIdx.z)
};

// Streaming accesses: every element of a pass is read once and written once, and
// the arrays (1-2 GB) are far larger than the caches.
template <class T> __device__ __forceinline__ C2<T> ld_stream(const C2<T>* p) {
  return {__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}
template <class T> __device__ __forceinline__ void st_stream(C2<T>* p, C2<T> v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// MODE 0: forward, 1: inverse.
// CONTIG: lines are contiguous (in_e == 1), batch = consecutive lines along o1;
// otherwise the batch is W = ELEMS/L adjacent lines (o1 stride 1) for coalescing.
// Batch size in elements: strided passes keep 16 adjacent complex64 lines (128-byte
// segments per row of the batch); contiguous passes take half, so that more
// workgroups fit the LDS of a compute unit.
template <class T, bool CONTIG> constexpr int batch_elems() { return (sizeof(T) == 4 && !CONTIG) ? 8192 : 4096; }

// HALF: a forward pass (MODE 0) whose lines are zero-padded to twice their length
// (n_in = L/2), or an inverse pass (MODE 1) that keeps the lower half (n_out = L/2).
template <class T, int L, bool CONTIG, int MODE, bool HALF>
__global__ void __launch_bounds__(kFftThreads) k_fft_pass(PassArgs a) {
  constexpr int ELEMS = batch_elems<T, CONTIG>();
  constexpr bool HIN = HALF && MODE == 0, HOUT = HALF && MODE == 1;
  constexpr int W = ELEMS / L;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  // complex64: twiddles staged in LDS; complex128: read from the (cached) table so
  // that two workgroups still fit the 160 KB of LDS of a compute unit
  constexpr bool TW_LDS = sizeof(T) == 4;
  C2<T>* tw_lds = lds + (ELEMS / L) * line_stride<L>();
  if (TW_LDS)
    for (int e = threadIdx.x; e < L; e += kFftThreads) tw_lds[e] = reinterpret_cast<const C2<T>*>(a.tw)[e];
  const C2<T>* tw = TW_LDS ? tw_lds : reinterpret_cast<const C2<T>*>(a.tw);
  const int g1 = blockIdx.x * W;     // first line along o1
  const int o2 = blockIdx.y;
  // Each thread owns PER elements of the batch.  All of its global loads are issued
  // before any is used (registers first, then LDS), so that PER requests per lane are
  // in flight instead of one.
  constexpr int PER = ELEMS / kFftThreads;
  static_assert(ELEMS % kFftThreads == 0, "batch not a multiple of the workgroup");
  auto coords = [&](int p, int& b, int& i) {
    const int e = threadIdx.x + p * kFftThreads;
    if (CONTIG) { b = e / L; i = e % L; } else { b = e % W; i = e / W; }
  };
  const int64_t in_o2 = boff(o2, a.in_o2, a.in_o2_hi, a.in_o2_sh);
  const int64_t out_o2 = boff(o2, a.out_o2, a.out_o2_hi, a.out_o2_sh);
  const C2<T>* in = reinterpret_cast<const C2<T>*>(a.in) + blockIdx.z * a.comp_in;
  C2<T>* out = reinterpret_cast<C2<T>*>(a.out) + blockIdx.z * a.comp_out;
  {
    C2<T> v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int b, i;
      coords(p, b, i);
      const int o1 = g1 + b;
      v[p] = {T(0), T(0)};
      if (o1 < a.n1 && i < a.n_in) v[p] = ld_stream(in + (o1 * a.in_o1 + in_o2 + boff(i, a.in_e, a.in_e_hi, a.in_e_sh)));
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int b, i;
      coords(p, b, i);
      if (!HIN || i < L / 2) lds[pidx<L>(b, i)] = v[p];   // the zero half is never read
    }
  }
  __syncthreads();
  fft_batch<T, L, ELEMS, MODE == 1, HIN, HOUT>(lds, tw);
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    int b, i;
    coords(p, b, i);
    const int o1 = g1 + b;
    if (o1 < a.n1 && i < a.n_out)
      st_stream(out + (o1 * a.out_o1 + out_o2 + boff(i, a.out_e, a.out_e_hi, a.out_e_sh)), lds[pidx<L>(b, i)]);
  }
}

// Fused z step of the free-space convolution: per batch of W adjacent (kx, ky) lines,
// forward FFT along z, product with the spectrum G^, inverse FFT, lower half kept.
// G^ is even in kz, so a batch reads its L/2 + 1 distinct values (z-pass layout
// [ky][kz][kx]: one strip per batch) and applies each to kz and L - kz.  Strided lines
// as in k_fft_pass (b = line in the batch, fastest).
//
// Workgroup order, XCD-aware: consecutive workgroups go to the eight XCDs in turn, each
// with an L2 of its own.  The workgroups that read the same G^ strip -- the components
// of one batch, the batch whose kx lines mirror it (kx and 2h - kx), and the line
// whose ky mirrors this one -- get ids that are multiples of eight apart (one XCD) and
// close in dispatch order, so that the strip comes from HBM once and from L2 after.
// In complex128 the strip is loaded with the lines, before the forward transform, which
// hides its latency; holding it across the transform must keep four waves per SIMD (at
// most 128 VGPRs), which the complex64 kernels (twice the lines per batch) and the
// 1024-point ones would exceed: they load it after the forward transform.
template <class T, int L> constexpr bool early_spectrum() { return sizeof(T) == 8 && L < 1024; }

template <class T, int L>
__global__ void __launch_bounds__(kFftThreads) k_fft_zconv(PassArgs a, int ncomp) {
  constexpr int ELEMS = batch_elems<T, false>();
  constexpr int W = ELEMS / L;
  constexpr int PER = ELEMS / kFftThreads;
  constexpr int NPAIR = W * (L / 2 + 1);
  constexpr int PG = (NPAIR + kFftThreads - 1) / kFftThreads;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  constexpr bool TW_LDS = sizeof(T) == 4;
  C2<T>* tw_lds = lds + W * line_stride<L>();
  if (TW_LDS)
    for (int e = threadIdx.x; e < L; e += kFftThreads) tw_lds[e] = reinterpret_cast<const C2<T>*>(a.tw)[e];
  const C2<T>* tw = TW_LDS ? tw_lds : reinterpret_cast<const C2<T>*>(a.tw);
  // batch and component: with nb % 16 == 0 (grid x a multiple of 8, so the XCD of a
  // workgroup is blockIdx.x % 8 on every grid row), XCD s holds, in dispatch order, the
  // batches s, nb-1-s, 8+s, nb-9-s, ..., each with all of its components
  const int nb = int(gridDim.x) / ncomp;
  int comp, batch;
  if (nb % 16 == 0) {
    const int xs = int(blockIdx.x % 8u), t = int(blockIdx.x / 8u);
    comp = t % ncomp;
    const int u = t / ncomp, base = 8 * (u / 2) + xs;
    batch = (u & 1) ? nb - 1 - base : base;
  } else {
    comp = int(blockIdx.x % unsigned(ncomp));
    batch = int(blockIdx.x / unsigned(ncomp));
  }
  // line o2: grid rows 2k-1 and 2k take ky = k and its mirror 2h - k (the same G^ row)
  int o2 = int(blockIdx.y);
  if (2 * a.h_o2 == int(gridDim.y) && o2 > 0) o2 = (o2 & 1) ? (o2 + 1) / 2 : int(gridDim.y) - o2 / 2;
  const int g1 = batch * W;
  const C2<T>* in = reinterpret_cast<const C2<T>*>(a.in) + comp * a.comp_in;
  C2<T>* out = reinterpret_cast<C2<T>*>(a.out) + comp * a.comp_out;
  const int64_t in_o2 = boff(o2, a.in_o2, a.in_o2_hi, a.in_o2_sh);
  const int64_t out_o2 = boff(o2, a.out_o2, a.out_o2_hi, a.out_o2_sh);
  // G^ strip: pair task t = (line b = t % W, kz = t / W), kz in [0, L/2]
  C2<T> gv[PG];
  auto load_spectrum = [&]() {
    const int m2 = o2 <= a.h_o2 ? o2 : 2 * a.h_o2 - o2;
    const C2<T>* G = reinterpret_cast<const C2<T>*>(a.mul) + int64_t(m2) * a.mul_o2;
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      const int t = threadIdx.x + p * kFftThreads, b = t % W, kz = t / W, o1 = g1 + b;
      const int m1 = o1 <= a.h_o1 ? o1 : 2 * a.h_o1 - o1;
      gv[p] = {T(0), T(0)};
      if (t < NPAIR && o1 < a.n1) gv[p] = G[int64_t(m1) * a.mul_o1 + int64_t(kz) * a.mul_e];
    }
  };
  {
    C2<T> v[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * kFftThreads, b = e % W, i = e / W, o1 = g1 + b;
      v[p] = {T(0), T(0)};
      if (o1 < a.n1 && i < a.n_in) v[p] = ld_stream(in + (o1 * a.in_o1 + in_o2 + boff(i, a.in_e, a.in_e_hi, a.in_e_sh)));
    }
    if (early_spectrum<T, L>()) load_spectrum();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * kFftThreads;
      if (e / W < L / 2) lds[pidx<L>(e % W, e / W)] = v[p];   // zero-padded upper half: never read
    }
  }
  __syncthreads();
  fft_batch<T, L, ELEMS, false, true, false>(lds, tw);
  if (!early_spectrum<T, L>()) load_spectrum();
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    const int t = threadIdx.x + p * kFftThreads, b = t % W, kz = t / W;
    if (t < NPAIR) {
      lds[pidx<L>(b, kz)] = cmul(lds[pidx<L>(b, kz)], gv[p]);
      if (kz > 0 && kz < L / 2) lds[pidx<L>(b, L - kz)] = cmul(lds[pidx<L>(b, L - kz)], gv[p]);
    }
  }
  __syncthreads();
  fft_batch<T, L, ELEMS, true, false, true>(lds, tw);   // the lower half is kept
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * kFftThreads, b = e % W, i = e / W, o1 = g1 + b;
    if (o1 < a.n1 && i < a.n_out)
      st_stream(out + (o1 * a.out_o1 + out_o2 + boff(i, a.out_e, a.out_e_hi, a.out_e_sh)), lds[pidx<L>(b, i)]);
  }
}

template <class T>
void launch_zconv_L(int L, const PassArgs& a, int ncomp, hipStream_t s) {
  SLIM_REQUIRE(2 * a.n_in == L && 2 * a.n_out == L, SLIM_E_STATE, "fused z pass: lines must be zero-padded to 2 Nz");
  constexpr int ELEMS = batch_elems<T, false>();
  const size_t shm = size_t((ELEMS / L) * (L + L / 8 + 1) + (sizeof(T) == 4 ? L : 0)) * sizeof(C2<T>);
  const int W = ELEMS / L;
  dim3 grid(unsigned((a.n1 + W - 1) / W * ncomp), unsigned(a.n2), 1u);
  switch (L) {
#define SLIM_ZCONV_CASE(LL)                                                                                   \
  case LL: {                                                                                                  \
    static bool attr_set = false;                                                                             \
    if (!attr_set) {                                                                                          \
      SLIM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_zconv<T, LL>),                        \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)));                     \
      attr_set = true;                                                                                        \
    }                                                                                                         \
    hipLaunchKernelGGL((k_fft_zconv<T, LL>), grid, dim3(kFftThreads), shm, s, a, ncomp);                      \
    break;                                                                                                    \
  }
    SLIM_ZCONV_CASE(16) SLIM_ZCONV_CASE(32) SLIM_ZCONV_CASE(64) SLIM_ZCONV_CASE(128) SLIM_ZCONV_CASE(256)
    SLIM_ZCONV_CASE(512) SLIM_ZCONV_CASE(1024)
#undef SLIM_ZCONV_CASE
    default: throw Error(SLIM_E_UNSUPPORTED, "FFT length " + std::to_string(L) + " (2N must be a power of two in [16, 1024])");
  }
  SLIM_HIP(hipGetLastError());
}

template <class T, bool CONTIG, int MODE, bool HALF>
void launch_pass_LH(int L, const PassArgs& a, int ncomp, hipStream_t s) {
  constexpr int ELEMS = batch_elems<T, CONTIG>();
  const size_t shm = size_t((ELEMS / L) * (L + L / 8 + 1) + (sizeof(T) == 4 ? L : 0)) * sizeof(C2<T>);
  const int W = ELEMS / L;
  dim3 grid(unsigned((a.n1 + W - 1) / W), unsigned(a.n2), unsigned(ncomp));
  switch (L) {
#define SLIM_FFT_CASE(LL)                                                                                   \
  case LL: {                                                                                                  \
    static bool attr_set = false;                                                                             \
    if (!attr_set) { /* more than 64 KB of dynamic LDS needs the explicit limit */                            \
      SLIM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_pass<T, LL, CONTIG, MODE, HALF>),     \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)));                     \
      attr_set = true;                                                                                        \
    }                                                                                                         \
    hipLaunchKernelGGL((k_fft_pass<T, LL, CONTIG, MODE, HALF>), grid, dim3(kFftThreads), shm, s, a);          \
    break;                                                                                                    \
  }
    SLIM_FFT_CASE(16) SLIM_FFT_CASE(32) SLIM_FFT_CASE(64) SLIM_FFT_CASE(128) SLIM_FFT_CASE(256)
    SLIM_FFT_CASE(512) SLIM_FFT_CASE(1024)
#undef SLIM_FFT_CASE
    default: throw Error(SLIM_E_UNSUPPORTED, "FFT length " + std::to_string(L) + " (2N must be a power of two in [16, 1024])");
  }
  SLIM_HIP(hipGetLastError());
}

// Pruned form when the lines are zero-padded to L (forward) or only their lower half is
// kept (inverse), as in every pass of the convolution; full transforms otherwise.
template <class T, bool CONTIG, int MODE>
void launch_pass_L(int L, const PassArgs& a, int ncomp, hipStream_t s) {
  const bool half = MODE == 0 ? 2 * a.n_in == L : 2 * a.n_out == L;
  if (half) launch_pass_LH<T, CONTIG, MODE, true>(L, a, ncomp, s);
  else launch_pass_LH<T, CONTIG, MODE, false>(L, a, ncomp, s);
}

// Spectrum product of the layered medium on the full-z spectra of the four
// components (lay: [comp][Z2][Y2][X2]), in place.  The reflected kernels depend on
// z + z', so they multiply the source spectrum at -kz; each thread takes the pair
// (kz, Z2 - kz) and writes both.  G^ (free space) is the even octant [ky][kz][kx]; the reflected
// spectra cover kx <= Nx, ky <= Ny (mirrored; zx odd in x, zy odd in y) and all kz.
template <class T>
__global__ void k_layered_mix(C2<T>* S, int64_t comp, const C2<T>* gp, const C2<T>* rh, int64_t spec, int Nx, int Ny,
                              int Nz, int do_vec, int do_rho) {
  const int X2 = 2 * Nx, Y2 = 2 * Ny, Z2 = 2 * Nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t plane = int64_t(X2) * Y2;
  if (i >= plane * (Nz + 1)) return;
  const int kx = int(i % X2), ky = int((i / X2) % Y2), k1 = int(i / plane);
  const int k2 = (Z2 - k1) % Z2;
  const int mx = kx <= Nx ? kx : X2 - kx, my = ky <= Ny ? ky : Y2 - ky;
  const T sx = kx <= Nx ? T(1) : T(-1), sy = ky <= Ny ? T(1) : T(-1);
  const int64_t o1 = int64_t(k1) * plane + int64_t(ky) * X2 + kx, o2 = int64_t(k2) * plane + int64_t(ky) * X2 + kx;
  // the vector components (0..2) and the charge (3) are independent products; a call
  // may take either set (they then run on different streams)
  C2<T> a[4], b[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const bool use = c < 3 ? do_vec : do_rho;
    a[c] = use ? S[c * comp + o1] : C2<T>{T(0), T(0)};
    b[c] = use ? S[c * comp + o2] : C2<T>{T(0), T(0)};
  }
  auto product = [&](int kz, const C2<T>* self, const C2<T>* part, C2<T>* r) {
    const int mz = kz <= Nz ? kz : Z2 - kz;
    const C2<T> g = gp[(int64_t(my) * (Nz + 1) + mz) * (Nx + 1) + mx];   // [ky][kz][kx]
    const int64_t ro = (int64_t(kz) * (Ny + 1) + my) * (Nx + 1) + mx;
    const C2<T> xx = rh[ro], zz = rh[spec + ro], ph = rh[2 * spec + ro];
    C2<T> zx = rh[3 * spec + ro], zy = rh[4 * spec + ro];
    zx = {sx * zx.x, sx * zx.y};
    zy = {sy * zy.x, sy * zy.y};
    // G_xz = -G_zx, G_yz = -G_zy
    r[0] = csub(cadd(cmul(g, self[0]), cmul(xx, part[0])), cmul(zx, part[2]));
    r[1] = csub(cadd(cmul(g, self[1]), cmul(xx, part[1])), cmul(zy, part[2]));
    r[2] = cadd(cadd(cmul(g, self[2]), cmul(zz, part[2])), cadd(cmul(zx, part[0]), cmul(zy, part[1])));
    r[3] = cadd(cmul(g, self[3]), cmul(ph, part[3]));
  };
  C2<T> r1[4], r2[4];
  product(k1, a, b, r1);
  product(k2, b, a, r2);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c < 3 ? !do_vec : !do_rho) continue;
    S[c * comp + o1] = r1[c];
    S[c * comp + o2] = r2[c];
  }
}

}  // namespace

void fft_init_twiddles(Ctx& c) {
  // three tables (one per axis), each of length 2 N_c
  std::vector<double> t128;
  std::vector<float> t64;
  for (int ax = 0; ax < 3; ++ax) {
    const int L = 2 * c.grid.N[ax];
    SLIM_REQUIRE(L >= 16 && L <= 1024 && (L & (L - 1)) == 0, SLIM_E_UNSUPPORTED,
                 "AIM grid size must be a power of two between 8 and 512 per axis");
    for (int m = 0; m < L; ++m) {
      double ang = -2.0 * kPi * double(m) / double(L);
      t128.push_back(std::cos(ang));
      t128.push_back(std::sin(ang));
      t64.push_back(float(std::cos(ang)));
      t64.push_back(float(std::sin(ang)));
    }
  }
  c.d_tw128.upload(t128);
  c.d_tw64.upload(t64);
}

static size_t tw_off(const Ctx& c, int ax) {
  size_t o = 0;
  for (int k = 0; k < ax; ++k) o += size_t(2 * c.grid.N[k]);
  return o;
}

void fft_forward_3d_c128(Ctx& c, double* data, hipStream_t s) {
  const int X2 = 2 * c.grid.N[0], Y2 = 2 * c.grid.N[1], Z2 = 2 * c.grid.N[2];
  const C2<double>* tw = c.d_tw128.as<C2<double>>();
  PassArgs a{};
  a.in = data; a.out = data; a.comp_in = a.comp_out = 0;
  // x: lines (y, z), contiguous
  a.in_e = a.out_e = 1; a.in_o1 = a.out_o1 = X2; a.in_o2 = a.out_o2 = int64_t(X2) * Y2;
  a.n1 = Y2; a.n2 = Z2; a.n_in = a.n_out = X2; a.tw = tw + tw_off(c, 0);
  launch_pass_L<double, true, 0>(X2, a, 1, s);
  // y: lines (x, z), stride X2
  a.in_e = a.out_e = X2; a.in_o1 = a.out_o1 = 1; a.in_o2 = a.out_o2 = int64_t(X2) * Y2;
  a.n1 = X2; a.n2 = Z2; a.n_in = a.n_out = Y2; a.tw = tw + tw_off(c, 1);
  launch_pass_L<double, false, 0>(Y2, a, 1, s);
  // z: lines (x, y), stride X2 Y2
  a.in_e = a.out_e = int64_t(X2) * Y2; a.in_o1 = a.out_o1 = 1; a.in_o2 = a.out_o2 = X2;
  a.n1 = X2; a.n2 = Y2; a.n_in = a.n_out = Z2; a.tw = tw + tw_off(c, 2);
  launch_pass_L<double, false, 0>(Z2, a, 1, s);
}

// Components [comp0, comp0 + ncomp) of oct_in (4 x N^3, [z][y][x]) -> oct_out, each
// convolved with the grid Green's function.  Distinct components use disjoint
// parts of every work array, so two calls on different components may run
// concurrently.
static void convolve_impl(Ctx& c, bool fp64, int ncomp, hipStream_t s, int comp0, bool layered) {
  const int Nx = c.grid.N[0], Ny = c.grid.N[1], Nz = c.grid.N[2];
  const int X2 = 2 * Nx, Y2 = 2 * Ny, Z2 = 2 * Nz;
  const int64_t N3 = c.grid.nodes();
  const size_t esz = fp64 ? 16 : 8;
  char* oin = reinterpret_cast<char*>(fp64 ? c.d_oct_in.p : c.d_oct_in32.p) + size_t(comp0) * N3 * esz;
  char* oout = reinterpret_cast<char*>(c.d_oct_out.p) + size_t(comp0) * N3 * esz;
  // z-block layout of the y-transformed array X2: planes are interleaved row by row in
  // blocks of B = 2^zsh planes, [z / B][y][z % B][x], so that a z line crosses Nz / B
  // blocks of B Y2 X2 elements instead of Nz planes of Y2 X2 elements (fewer pages per
  // line); B = 1 is the plain [z][y][x] order
  const int zsh = c.fft_zsh;
  const int64_t ZLO = zsh ? int64_t(X2) : int64_t(X2) * Y2, ZHI = int64_t(X2) * Y2 << zsh, YST = int64_t(X2) << zsh;
  const int64_t CS2 = 4 * N3;
  char* x1 = reinterpret_cast<char*>(c.d_x1.p) + size_t(comp0) * 2 * N3 * esz;
  char* x2 = reinterpret_cast<char*>(c.d_x2.p) + size_t(comp0) * CS2 * esz;
  auto z_axis_in = [&](PassArgs& a) { a.in_e = ZLO; a.in_e_hi = ZHI; a.in_e_sh = zsh; };
  auto z_axis_out = [&](PassArgs& a) { a.out_e = ZLO; a.out_e_hi = ZHI; a.out_e_sh = zsh; };
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const C2<T>* tw = reinterpret_cast<const C2<T>*>(fp64 ? c.d_tw128.p : c.d_tw64.p);
    PassArgs a{};
    // x-fwd: octant [Nz][Ny][Nx] -> X1 [Nz][Ny][X2]
    a.in = oin; a.out = x1;
    a.in_e = 1; a.in_o1 = Nx; a.in_o2 = int64_t(Nx) * Ny;
    a.out_e = 1; a.out_o1 = X2; a.out_o2 = int64_t(X2) * Ny;
    a.n1 = Ny; a.n2 = Nz; a.n_in = Nx; a.n_out = X2;
    a.comp_in = N3; a.comp_out = 2 * N3;
    a.tw = tw + tw_off(c, 0);
    launch_pass_L<T, true, 0>(X2, a, ncomp, s);
    // y-fwd: X1 [Nz][Ny][X2] -> X2 [Nz][Y2][X2]
    a = PassArgs{};
    a.in = x1; a.out = x2;
    a.in_e = X2; a.in_o1 = 1; a.in_o2 = int64_t(X2) * Ny;
    a.out_e = YST; a.out_o1 = 1; a.out_o2 = ZLO; a.out_o2_hi = ZHI; a.out_o2_sh = zsh;
    a.n1 = X2; a.n2 = Nz; a.n_in = Ny; a.n_out = Y2;
    a.comp_in = 2 * N3; a.comp_out = CS2;
    a.tw = tw + tw_off(c, 1);
    launch_pass_L<T, false, 0>(Y2, a, ncomp, s);
    if (!layered) {
      // z fused: X2 lines (kx, ky), stride X2 Y2; forward, x G^, inverse, keep z < Nz
      a = PassArgs{};
      a.in = x2; a.out = x2;
      z_axis_in(a); z_axis_out(a); a.in_o1 = a.out_o1 = 1; a.in_o2 = a.out_o2 = YST;
      a.n1 = X2; a.n2 = Y2; a.n_in = Nz; a.n_out = Nz;
      a.mul = fp64 ? c.d_ghat128.p : c.d_ghat64.p;   // [ky][kz][kx]
      a.mul_o1 = 1; a.mul_e = Nx + 1; a.mul_o2 = int64_t(Nx + 1) * (Nz + 1);
      a.h_e = Nz; a.h_o1 = Nx; a.h_o2 = Ny;
      a.comp_in = a.comp_out = CS2;
      a.tw = tw + tw_off(c, 2);
      launch_zconv_L<T>(Z2, a, ncomp, s);
    } else {
      // layered z step: forward into the full-z work array, spectrum product with
      // the partner -kz, inverse back (keep z < Nz)
      SLIM_REQUIRE((comp0 == 0 && (ncomp == 3 || ncomp == 4)) || (comp0 == 3 && ncomp == 1), SLIM_E_ARG,
                   "layered convolution takes the vector components, the charge, or all four");
      char* lay0 = reinterpret_cast<char*>(c.d_lay.p);
      char* lay = lay0 + size_t(comp0) * 8 * N3 * esz;
      a = PassArgs{};
      a.in = x2; a.out = lay;
      z_axis_in(a); a.out_e = int64_t(X2) * Y2; a.in_o1 = a.out_o1 = 1; a.in_o2 = YST; a.out_o2 = X2;
      a.n1 = X2; a.n2 = Y2; a.n_in = Nz; a.n_out = Z2;
      a.comp_in = CS2; a.comp_out = 8 * N3;
      a.tw = tw + tw_off(c, 2);
      launch_pass_L<T, false, 0>(Z2, a, ncomp, s);
      const int64_t pairs = int64_t(X2) * Y2 * (Nz + 1);
      const int64_t spec = int64_t(Nx + 1) * (Ny + 1) * Z2;
      hipLaunchKernelGGL((k_layered_mix<T>), dim3(unsigned((pairs + 255) / 256)), dim3(256), 0, s,
                         reinterpret_cast<C2<T>*>(lay0), 8 * N3,
                         reinterpret_cast<const C2<T>*>(fp64 ? c.d_ghat128.p : c.d_ghat64.p),
                         reinterpret_cast<const C2<T>*>(fp64 ? c.d_rhat128.p : c.d_rhat64.p), spec, Nx, Ny, Nz,
                         comp0 == 0 ? 1 : 0, comp0 + ncomp == 4 ? 1 : 0);
      SLIM_HIP(hipGetLastError());
      a = PassArgs{};
      a.in = lay; a.out = x2;
      a.in_e = int64_t(X2) * Y2; z_axis_out(a); a.in_o1 = a.out_o1 = 1; a.in_o2 = X2; a.out_o2 = YST;
      a.n1 = X2; a.n2 = Y2; a.n_in = Z2; a.n_out = Nz;
      a.comp_in = 8 * N3; a.comp_out = CS2;
      a.tw = tw + tw_off(c, 2);
      launch_pass_L<T, false, 1>(Z2, a, ncomp, s);
    }
    // y-inv: X2 [Nz][Y2][X2] -> X1 [Nz][Ny][X2] (keep y < Ny)
    a = PassArgs{};
    a.in = x2; a.out = x1;
    a.in_e = YST; a.in_o1 = 1; a.in_o2 = ZLO; a.in_o2_hi = ZHI; a.in_o2_sh = zsh;
    a.out_e = X2; a.out_o1 = 1; a.out_o2 = int64_t(X2) * Ny;
    a.n1 = X2; a.n2 = Nz; a.n_in = Y2; a.n_out = Ny;
    a.comp_in = CS2; a.comp_out = 2 * N3;
    a.tw = tw + tw_off(c, 1);
    launch_pass_L<T, false, 1>(Y2, a, ncomp, s);
    // x-inv: X1 [Nz][Ny][X2] -> octant (keep x < Nx)
    a = PassArgs{};
    a.in = x1; a.out = oout;
    a.in_e = 1; a.in_o1 = X2; a.in_o2 = int64_t(X2) * Ny;
    a.out_e = 1; a.out_o1 = Nx; a.out_o2 = int64_t(Nx) * Ny;
    a.n1 = Ny; a.n2 = Nz; a.n_in = X2; a.n_out = Nx;
    a.comp_in = 2 * N3; a.comp_out = N3;
    a.tw = tw + tw_off(c, 0);
    launch_pass_L<T, true, 1>(X2, a, ncomp, s);
  };
  if (fp64) run(double{});
  else run(float{});
}

void aim_convolve(Ctx& c, bool fp64, int ncomp, hipStream_t s, int comp0, bool layered) {
  SLIM_REQUIRE(!layered || c.layered, SLIM_E_STATE, "no layered medium set");
  convolve_impl(c, fp64, ncomp, s, comp0, layered);
}

// The four components over a layered background (free-space kernel plus the
// reflected dyadic); needs build_layered.
void aim_convolve_layered(Ctx& c, bool fp64, hipStream_t s) {
  SLIM_REQUIRE(c.layered, SLIM_E_STATE, "no layered medium set");
  convolve_impl(c, fp64, 4, s, 0, true);
}

}  // namespace slim
