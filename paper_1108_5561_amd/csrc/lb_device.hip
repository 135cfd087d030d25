// Device kernels of the Milne quasiparticle lattice-Boltzmann step for
// gfx950 (paper Sec. IV.D, eqs. (Bmilne), (newBeq), (bgk), (sanity),
// (emtnew), (masschange)).
//
// Work mapping: eight lanes per lattice site, lane l owning the phi_l slice
// (N_xi x N_theta nodes) of that site.  The weak-form operators S1, S2 act
// within one phi slice, so they are lane-local; the moments and the mass
// evolution sums are reduced over the eight lanes with DPP moves (sum8:
// all lanes end with bitwise-identical sums).  The per-site FP64 matching
// of a state runs once per site, in the first wave of the block that
// produced the state (match_moments, match_sites).
//
// Distribution layout in HBM (NodeLayout): the 25 nodes of a slice in
// 16-byte groups, group g in plane g as [site][l][V], so a lane moves its
// slice with a few 16-byte loads and a wave (8 sites x 8 slices) reads and
// writes 1 KB contiguous per group.
#include <hip/hip_runtime.h>

#include "../../include/lb.h"
#include "device_common.hpp"
#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

constexpr int kSl = 8;        // phi slices (n_phi = 4)
constexpr int kBlock = 256;   // 32 sites per block

// ---------------------------------------------------------------------------
// One Heun stage (Sec. IV.D).  STAGE 0 = predictor, 1 = corrector.
//
// A block owns an 8 x TY tile of sites (8 lanes per site, lane l owning the
// phi_l slice).  The per-site FP64 work of a state (Landau matching of
// eq. (sanity), EoS inversion) is done once, at the end of the kernel that
// produced the state, and handed to the next stage as per-site scalars.  A
// stage therefore has no wait on it:
//  1. load the site scalars of the input state, the slice and its upwind
//     neighbours; streaming, Milne term S1/tau, S2;
//  2. equilibrium, BGK, mass-gradient force, the mass-evolution sums, X and
//     the Heun update, stored;
//  3. moments of the new state (eq. (emtnew)), reduced over the eight slices;
//     one barrier; the first wave matches them (one lane per site, FP64) and
//     writes the site scalars of the new state.
//
// Polar mirror pairs: the node set is symmetric under theta -> pi - theta
// (j -> 4 - j), and the equilibrium, |v_perp|, gamma and the weights are
// even under it, so per slice those are evaluated on 15 (k, pair) values
// and shared by the two nodes of a pair; the polar part of S1 is applied in
// the mirror-even / mirror-odd basis.
constexpr int kTX = 8;
constexpr int kXcds = 8;  // accelerator complex dies of the MI355X
constexpr size_t kMallBytes = (size_t)192 << 20;  // below the 256 MB last-level cache
constexpr int kBigTileRows = 8;
// rows of the per-tile moment exchange: T^{ab} (6), ln M, N^a (3, mu mode)
constexpr int kMomRows = 10;
#ifndef LB_TILE_ROWS_F32
#define LB_TILE_ROWS_F32 4
#endif
#ifndef LB_WAVES_PER_EU_F32
#define LB_WAVES_PER_EU_F32 4
#endif
#ifndef LB_WAVES_PER_EU_F64
#define LB_WAVES_PER_EU_F64 2
#endif
template <typename R> struct TileRows { static constexpr int v = LB_TILE_ROWS_F32; };
template <> struct TileRows<double> { static constexpr int v = 4; };
#ifndef LB_WAVES_PER_EU_F32_CORR
#define LB_WAVES_PER_EU_F32_CORR LB_WAVES_PER_EU_F32
#endif
template <typename R, int STAGE> struct MinWaves {
  static constexpr int v = STAGE == 0 ? LB_WAVES_PER_EU_F32 : LB_WAVES_PER_EU_F32_CORR;
};
// FP64: the predictor at one wave per SIMD (65 us against 72 at two, whose
// register budget makes it spill), the corrector at two (89 us against 138)
#ifndef LB_WAVES_PER_EU_F64_PRED
#define LB_WAVES_PER_EU_F64_PRED 1
#endif
template <int STAGE> struct MinWaves<double, STAGE> {
  static constexpr int v = STAGE == 0 ? LB_WAVES_PER_EU_F64_PRED : LB_WAVES_PER_EU_F64;
};
// with the weak-form 3-D force (about twice the registers in flight)
#ifndef LB_FORCE_WAVES_F32
#define LB_FORCE_WAVES_F32 2
#endif
template <typename R> struct ForceWaves { static constexpr int v = LB_FORCE_WAVES_F32; };
template <> struct ForceWaves<double> { static constexpr int v = 1; };
// with the conserved particle number (the n matching's registers)
template <typename R> struct MuWaves { static constexpr int v = 3; };
template <> struct MuWaves<double> { static constexpr int v = LB_WAVES_PER_EU_F64; };

// A distribution buffer is read and written as one raw buffer: one
// descriptor (uniform, scalar registers), the plane offset q * plane bytes
// as the scalar offset and a 32-bit byte offset per lane, so no per-load
// vector address arithmetic.  Out-of-range offsets read 0 and drop writes;
// the host keeps a buffer below 4 GiB.
typedef unsigned lb_v2u __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename R> struct Buf;
// kAux is the cache-policy operand of the buffer instruction: 0, kNT
// (nontemporal: the line is not kept for reuse, for data streamed once) or
// kSC1 (device scope: a store is written through this XCD's L2 to the
// memory side, where the next stage's blocks on every XCD read it)
constexpr int kNT = 2;
constexpr int kSC1 = 16;
template <> struct Buf<float> {
  template <int kAux = 0>
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, kAux));
  }
  template <int kAux = 0>
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, (int)soff, kAux);
  }
};
template <> struct Buf<double> {
  template <int kAux = 0>
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, kAux));
  }
  template <int kAux = 0>
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(lb_v2u, v), r, (int)off, (int)soff, kAux);
  }
};

// 16-byte vector access (dwordx4): one instruction moves V = 16 / sizeof(R)
// values of a lane.
typedef unsigned lb_v4u __attribute__((ext_vector_type(4)));
template <typename R, int kAux = 0>
__device__ __forceinline__ void ld_vec(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, R* out) {
  // the whole vector is reinterpreted at once (a bit cast of a single
  // vector element is not used: it does not survive the load narrowing)
  typedef R lb_vr __attribute__((ext_vector_type(16 / sizeof(R))));
  const lb_vr v = __builtin_bit_cast(lb_vr, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)soff, kAux));
#pragma unroll
  for (int i = 0; i < (int)(16 / sizeof(R)); ++i) out[i] = v[i];
}
template <typename R, int kAux = 0>
__device__ __forceinline__ void st_vec(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, const R* in) {
  typedef R lb_vr __attribute__((ext_vector_type(16 / sizeof(R))));
  lb_vr v;
#pragma unroll
  for (int i = 0; i < (int)(16 / sizeof(R)); ++i) v[i] = in[i];
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(lb_v4u, v), r, (int)off, (int)soff, kAux);
}

// Distribution layout in HBM.  The 25 nodes q = k N_theta + j of a slice
// (site, l) are stored in groups of V = 16 / sizeof(R) consecutive nodes,
// group g = q / V in plane g as [site][l][V]; the last node (q = 24) in a
// plane of its own, [site][l].  A lane moves its slice with 24 / V + 1
// instructions, a wavefront (8 sites x 8 slices) 1 KB per group.
template <typename R>
struct NodeLayout {
  static constexpr int V = 16 / (int)sizeof(R);
  static constexpr int NG = 24 / V;  // full groups
  // bytes of one group plane
  static __device__ __host__ uint32_t gbytes(int n_sites) { return (uint32_t)n_sites * kSl * 16u; }
  // byte offset of node q of slice (site, l)
  static __device__ __host__ size_t offset(int q, int site, int l, int n_sites) {
    const size_t lane = (size_t)site * kSl + l;
    if (q < NG * V) return (size_t)(q / V) * gbytes(n_sites) + (lane * V + (size_t)(q % V)) * sizeof(R);
    return (size_t)NG * gbytes(n_sites) + lane * sizeof(R);
  }
};

// Slice of lane index lane = site * 8 + l: load / store all 25 nodes.
template <typename R, int kAux = 0>
__device__ __forceinline__ void load_slice(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t gb, R f[25]) {
  using L = NodeLayout<R>;
#pragma unroll
  for (int g = 0; g < L::NG; ++g) ld_vec<R, kAux>(r, lane * 16u, g * gb, &f[g * L::V]);
  f[24] = Buf<R>::template ld<kAux>(r, lane * (uint32_t)sizeof(R), L::NG * gb);
}
template <typename R, int kAux = 0>
__device__ __forceinline__ void store_slice(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t gb, const R f[25]) {
  using L = NodeLayout<R>;
#pragma unroll
  for (int g = 0; g < L::NG; ++g) st_vec<R, kAux>(r, lane * 16u, g * gb, &f[g * L::V]);
  Buf<R>::template st<kAux>(r, lane * (uint32_t)sizeof(R), L::NG * gb, f[24]);
}

// Site record (kernels.hpp): kScN values of R, then beta and ln M (FP64).
template <typename R>
struct SiteRecord {
  static constexpr uint32_t kBytes = kScN * (uint32_t)sizeof(R) + 16u;
  static constexpr int kVecs = (int)(kBytes / 16u);
  R v[kScN];
  double beta, lnM;
};
template <typename R>
__device__ __forceinline__ SiteRecord<R> load_record(__amdgpu_buffer_rsrc_t r, int site) {
  SiteRecord<R> rec;
  R w[SiteRecord<R>::kVecs * NodeLayout<R>::V];
#pragma unroll
  for (int i = 0; i < SiteRecord<R>::kVecs; ++i)
    ld_vec<R>(r, (uint32_t)site * SiteRecord<R>::kBytes + 16u * i, 0, &w[i * NodeLayout<R>::V]);
#pragma unroll
  for (int i = 0; i < kScN; ++i) rec.v[i] = w[i];
  if constexpr (sizeof(R) == 4) {
    rec.beta = __builtin_bit_cast(double, (uint64_t)__builtin_bit_cast(unsigned, w[kScN]) |
                                              ((uint64_t)__builtin_bit_cast(unsigned, w[kScN + 1]) << 32));
    rec.lnM = __builtin_bit_cast(double, (uint64_t)__builtin_bit_cast(unsigned, w[kScN + 2]) |
                                             ((uint64_t)__builtin_bit_cast(unsigned, w[kScN + 3]) << 32));
  } else {
    rec.beta = (double)w[kScN];
    rec.lnM = (double)w[kScN + 1];
  }
  return rec;
}
template <typename R>
__device__ __forceinline__ void store_record(__amdgpu_buffer_rsrc_t r, int site, const SiteRecord<R>& rec) {
  R w[SiteRecord<R>::kVecs * NodeLayout<R>::V];
#pragma unroll
  for (int i = 0; i < kScN; ++i) w[i] = rec.v[i];
  if constexpr (sizeof(R) == 4) {
    const uint64_t b = __builtin_bit_cast(uint64_t, rec.beta), m = __builtin_bit_cast(uint64_t, rec.lnM);
    w[kScN] = __builtin_bit_cast(R, (unsigned)b);
    w[kScN + 1] = __builtin_bit_cast(R, (unsigned)(b >> 32));
    w[kScN + 2] = __builtin_bit_cast(R, (unsigned)m);
    w[kScN + 3] = __builtin_bit_cast(R, (unsigned)(m >> 32));
  } else {
    w[kScN] = rec.beta;
    w[kScN + 1] = rec.lnM;
  }
#pragma unroll
  for (int i = 0; i < SiteRecord<R>::kVecs; ++i)
    st_vec<R>(r, (uint32_t)site * SiteRecord<R>::kBytes + 16u * i, 0, &w[i * NodeLayout<R>::V]);
}

// Node arithmetic helpers: hardware exp2 / sqrt / reciprocal in FP32 (about
// 1 ulp), the correctly rounded library functions in FP64.
template <typename R> __device__ __forceinline__ R eq_exp2(R a);
template <> __device__ __forceinline__ float eq_exp2<float>(float a) { return __builtin_amdgcn_exp2f(a); }
template <> __device__ __forceinline__ double eq_exp2<double>(double a) { return exp2(a); }
template <typename R> __device__ __forceinline__ R nsqrt(R a);
template <> __device__ __forceinline__ float nsqrt<float>(float a) { return __builtin_amdgcn_sqrtf(a); }
template <> __device__ __forceinline__ double nsqrt<double>(double a) { return sqrt(a); }
template <typename R> __device__ __forceinline__ R nrcp(R a);
template <> __device__ __forceinline__ float nrcp<float>(float a) { return __builtin_amdgcn_rcpf(a); }
template <> __device__ __forceinline__ double nrcp<double>(double a) { return 1.0 / a; }

// Stage constants live in device memory and are read with scalar loads
// through a constant-address-space pointer; const_ptr hides the pointer's
// value from the optimiser at the point of use, so a loop re-reads them
// instead of holding all of them in registers across iterations.
template <typename R>
using CPtr = const __attribute__((address_space(4))) StageConst<R>*;
template <typename R>
__device__ __forceinline__ CPtr<R> const_ptr(const StageConst<R>* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (CPtr<R>)v;
}
// The EoS table descriptor from its device copy, with scalar loads at the
// point of use.  Field by field: a field added to EosTable must be added
// here too (the size check below fails until it is).
static_assert(sizeof(EosTable) == 160, "EosTable changed: update load_table");
__device__ __forceinline__ EosTable load_table(const EosTable* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  const __attribute__((address_space(4))) EosTable* q = (const __attribute__((address_space(4))) EosTable*)v;
  EosTable t;
  t.pts = q->pts;
  t.inv_ek = q->inv_ek;
  t.inv_ee = q->inv_ee;
  t.n = q->n;
  t.n_inv = q->n_inv;
  t.u0 = q->u0;
  t.h = q->h;
  t.inv_h = q->inv_h;
  t.gk0 = q->gk0;
  t.gk_h = q->gk_h;
  t.gk_inv_h = q->gk_inv_h;
  t.ge0 = q->ge0;
  t.ge_h = q->ge_h;
  t.ge_inv_h = q->ge_inv_h;
  t.u_lo = q->u_lo;
  t.u_hi = q->u_hi;
  t.gpts = q->gpts;
  t.gn = q->gn;
  t.gpad_ = 0;
  t.gg0 = q->gg0;
  t.gg_h = q->gg_h;
  t.gg_inv_h = q->gg_inv_h;
  return t;
}
// Entry l (0..7, this lane's phi slice) of an 8-value table in the stage
// constants, two ways.  lane_load reads it per lane: the FP32 stage kernels
// issue these reads before their streaming loads, so that the in-order
// vector-memory counter lets the values be used without waiting for the
// loads issued after them.  lane_entry reads the table with scalar loads
// and selects the lane's value in registers (more instructions, no memory
// latency: the FP64 kernels, at one or two waves per SIMD, are faster so).
template <typename R>
__device__ __forceinline__ R lane_load(const __attribute__((address_space(4))) R* tab, int l) {
  return tab[l];
}
template <typename R>
__device__ __forceinline__ R lane_entry(const __attribute__((address_space(4))) R* tab, int l) {
  R v[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) v[d] = tab[d];
  R r = v[7];
#pragma unroll
  for (int d = 6; d >= 0; --d) r = (l == d) ? v[d] : r;
  return r;
}

// ---- weak-form 3-D mass-gradient force ---------------------------------
// Value of lane (lane ^ 1) (the cos/sin partner mode) of the 8-lane group.
template <typename R>
__device__ __forceinline__ R partner_lane(R v);
template <>
__device__ __forceinline__ float partner_lane<float>(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
template <>
__device__ __forceinline__ double partner_lane<double>(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0xB1, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The eight phi-slice values of node q of this lane's site from the wave's
// exchange area sw[25][64] (lane-in-wave order), two 16-byte reads per
// 4 values; the site's lanes read the same addresses (broadcast).
template <typename R>
__device__ __forceinline__ void site_values(const R* sw, int q, int sb, R v[8]) {
  constexpr int V = 16 / (int)sizeof(R);
  typedef R Vec __attribute__((ext_vector_type(V)));
  const Vec* p = reinterpret_cast<const Vec*>(sw + q * 64 + sb);
#pragma unroll
  for (int i = 0; i < 8 / V; ++i) {
    const Vec x = p[i];
#pragma unroll
    for (int c = 0; c < V; ++c) v[i * V + c] = x[c];
  }
}

// radial part of the transposed strong-form derivative for one mu column
// h[k] of a Fourier mode: odd (e = 1) for s P(x), even for P(x):
//   e = 0: r = Dx^T (s/x . h);   e = 1: r = (1/s) (Dx^T (s^2/x . h) + h)
template <typename R>
__device__ __forceinline__ void radial_t(const R h[5], bool e, CPtr<R> C, R r[5]) {
  R u[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) u[k] = (e ? C->frho1[k] : C->frho0[k]) * h[k];
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    R acc = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) acc += C->fDxT[b * 5 + k] * u[k];
    r[b] = e ? C->fsig1[b] * (acc + h[b]) : acc;
  }
}

// Adds scale * sum_i g_i G_i F to r0 for this lane's phi slice l, where G_i
// is the weak form of (1/gamma) [v^i (v . d_v) + d_{v^i}] on the test space
// of eq. (fansatz) (Sec. IV.B: harmonics of v/|v| of degree n = m + j,
// Fourier mode m in phi, times s^{n mod 2} P(cosh xi)).  Weak form: for
// every test function psi, sum w psi (G_i F) = sum w F b_i[psi] with
// b_i[psi] = -(1/gamma) [v^i (v . grad psi) + d_i psi + 2 v^i psi], which is
// minus the w-weighted transpose of the strong derivatives of the
// interpolant (StageConst::f* documents the factors).  The phi dependence
// goes through a real Fourier transform over the site's 8 lanes (lane r
// holds mode r after the analysis), exchanged through the wave's LDS area
// sw[25][64] (lw = lane in the wave); radial and polar derivatives act per
// mode; the synthesis brings the result back to phi slices.  Every thread
// of the block calls it (block barriers).
template <typename R>
__device__ __forceinline__ void weak_force(const R f[25], CPtr<R> C, R gx, R gy, int l, R scale, R r0[25], R* sw,
                                           int lw) {
  const int sb = lw & 56;  // first lane of this site in the wave
  const R cl = C->cosl[l], sl = C->sinl[l];
  const R gr = gx * cl + gy * sl;  // g . (cos phi, sin phi)
  // this lane's mode (as a mode index r = l): 0, 4, 1c, 1s, 2c, 2s, 3c, 3s
  const int m = l < 2 ? 4 * l : (l >> 1);
  const bool sine = l >= 2 && (l & 1);
  const bool modd = (m & 1) != 0;
  // d/dphi: cos m phi -> -m sin m phi, sin m phi -> m cos m phi; the
  // transpose takes -m times the sine partner into a cosine mode, +m times
  // the cosine partner into a sine mode (partners are lanes r and r ^ 1)
  const R dphi = l < 2 ? (R)0 : (sine ? (R)m : (R)(-m));

  R ph[25], out[25];
  // analysis of g_r w F and g_t w F (g_r = g . (cos, sin), g_t = g . (-sin,
  // cos)) from one exchange of F: with A_r = sum_l Phi_r(phi_l) cos(phi_l) F_l
  // and B_r the same with sin(phi_l), the modes are w (g_x A + g_y B) and
  // w (g_y A - g_x B)
#pragma unroll
  for (int q = 0; q < 25; ++q) sw[q * 64 + lw] = f[q];
  __syncthreads();
  {
    R ca[8], cb[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const R ph_ = C->fphi[d * 8 + l];
      ca[d] = ph_ * C->cosl[d];
      cb[d] = ph_ * C->sinl[d];
    }
#pragma unroll
    for (int q = 0; q < 25; ++q) {
      R v[8];
      site_values<R>(sw, q, sb, v);
      R A = 0, B = 0;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        A += ca[d] * v[d];
        B += cb[d] * v[d];
      }
      const R wq = C->fw[q];
      ph[q] = wq * (gx * A + gy * B);
      out[q] = dphi * partner_lane<R>(C->fc[q] * (wq * (gy * A - gx * B)));
    }
  }
  // radial: even and odd parts in mu carry s^{m mod 2} and s^{(m+1) mod 2}
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    R he[5], ho[5], re[5], ro[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int qa = k * 5 + pr, qb = k * 5 + 4 - pr;
      const R aa = C->fa[qa] * ph[qa];
      if (pr < 2) {
        const R ab = C->fa[qb] * ph[qb];
        he[k] = (R)0.5 * (aa + ab);
        ho[k] = (R)0.5 * (aa - ab);
      } else {
        he[k] = aa;
      }
    }
    radial_t<R>(he, modd, C, re);
    if (pr < 2) {
      radial_t<R>(ho, !modd, C, ro);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        out[k * 5 + pr] += re[k] + ro[k];
        out[k * 5 + 4 - pr] += re[k] - ro[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) out[k * 5 + 2] += re[k];
    }
  }
  // polar: similarity by (1 - mu^2)^{m/2} of the Legendre-node derivative
  {
    R pw0 = 1, pw1 = 1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < m) {
        pw0 *= C->fst[0];
        pw1 *= C->fst[1];
      }
    const R pw[5] = {pw0, pw1, (R)1, pw1, pw0};
    const R ipw0 = (R)1 / pw0, ipw1 = (R)1 / pw1;
    const R ipw[5] = {ipw0, ipw1, (R)1, ipw1, ipw0};
    const R mr = (R)m;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      R b[5], v[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        b[j] = C->fb[k * 5 + j] * ph[k * 5 + j];
        v[j] = pw[j] * b[j];
      }
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        R acc = 0;
#pragma unroll
        for (int jp = 0; jp < 5; ++jp) acc += C->fDmT[j * 5 + jp] * v[jp];
        out[k * 5 + j] += acc * ipw[j] - mr * C->fmr[j] * b[j];
      }
    }
  }
  // synthesis (1/sum_l Phi_r(phi_l)^2 folded into the coefficients) and the
  // undifferentiated term
  __syncthreads();  // every lane has read F
#pragma unroll
  for (int q = 0; q < 25; ++q) sw[q * 64 + lw] = out[q];
  __syncthreads();
  {
    R cs[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) cs[d] = C->fphi[l * 8 + d] * (d < 2 ? (R)0.125 : (R)0.25);
#pragma unroll
    for (int q = 0; q < 25; ++q) {
      R v[8];
      site_values<R>(sw, q, sb, v);
      R acc = 0;
#pragma unroll
      for (int d = 0; d < 8; ++d) acc += cs[d] * v[d];
      const R P = gr * C->fw[q] * f[q];
      r0[q] -= scale * C->finvw[q] * (acc + C->fy[q] * P);
    }
  }
}

// Dense form of the weak-form force operators, for the FP64 adjoint:
// G_i[n][m] = (G_i e_m)_n over the canonical node index n = q 8 + l, from
// weak_force applied to unit vectors, so that the adjoint differentiates
// the same operator as the stage kernels.  One wave per block: eight probe
// sites of eight slices, probe site = column m = 8 blockIdx.x + t / 8
// (gridDim.x = 25), component i = blockIdx.y (0: x, 1: y); G holds
// [2][200][200].
__global__ __launch_bounds__(64) void force_columns_kernel(const StageConst<double>* __restrict__ Cg,
                                                           double* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) double s_force[25 * 64];
  const int t = threadIdx.x, l = t & 7;
  const int m = (int)blockIdx.x * 8 + (t >> 3);
  const int comp = (int)blockIdx.y;
  const CPtr<double> C = const_ptr(Cg);
  double f[25], r0[25];
#pragma unroll
  for (int q = 0; q < 25; ++q) {
    f[q] = (q * 8 + l == m) ? 1.0 : 0.0;
    r0[q] = 0.0;
  }
  weak_force<double>(f, C, comp == 0 ? 1.0 : 0.0, comp == 1 ? 1.0 : 0.0, l, 1.0, r0, s_force, t);
  double* Gi = G + (size_t)comp * 200 * 200;
#pragma unroll
  for (int q = 0; q < 25; ++q) Gi[(size_t)(q * 8 + l) * 200 + m] = r0[q];
}

// Partial moments of one slice over the mirror pairs: w gamma^2, w gamma
// |v_perp|, w |v_perp|^2 and w, summed over the 25 nodes (eq. (emtnew)).
template <typename R>
__device__ __forceinline__ void slice_moments(const R f[25], CPtr<R> C, R* p0, R* p1, R* p2, R* p3) {
  R a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const R fs = pr < 2 ? f[k * 5 + pr] + f[k * 5 + 4 - pr] : f[k * 5 + 2];
      const int i = k * 3 + pr;
      a0 += C->wx2[i] * fs;
      a1 += C->wxs[i] * fs;
      a2 += C->ws2[i] * fs;
      a3 += C->w[i] * fs;
    }
  }
  *p0 = a0;
  *p1 = a1;
  *p2 = a2;
  *p3 = a3;
}

// Particle-current partial sums of one slice over the mirror pairs:
// w gamma and w |v_perp| (eq. (NTdisc)).
template <typename R>
__device__ __forceinline__ void slice_current(const R f[25], CPtr<R> C, R* p0, R* p1) {
  R a0 = 0, a1 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const R fs = pr < 2 ? f[k * 5 + pr] + f[k * 5 + 4 - pr] : f[k * 5 + 2];
      const int i = k * 3 + pr;
      a0 += C->w[i] * C->x[k] * fs;
      a1 += C->w[i] * C->sig[i] * fs;
    }
  }
  *p0 = a0;
  *p1 = a1;
}

// Landau matching (eq. (sanity)) and EoS inversion of a tile's state from
// the slices in registers, writing the site scalars, in two calls made by
// every thread of the block: match_moments puts the slice sums into LDS
// (lane l of site ts holds slice l, cl and sl are the cosine and sine of
// its angle, lnM = ln M of its site; s_mom is the block's LDS scratch
// [rows][tile sites]), match_sites waits at the block's barrier and has one
// thread per site match it and write its record.  A kernel may do other
// work (its stores) between the two.
template <typename R, int kTY, int kMu, bool kSelect = false>
__device__ __forceinline__ void match_moments(const R f[25], CPtr<R> C, R cl, R sl, double lnM, int t,
                                              double (*s_mom)[kTX * kTY]) {
  const int ts = t >> 3, l = t & 7;
  R p0, p1, p2, p3;
  slice_moments(f, C, &p0, &p1, &p2, &p3);
  (void)p3;
  if constexpr (kSelect) {  // the angles by lane_entry, here (cl, sl unused)
    cl = lane_entry<R>(C->cosl, l);
    sl = lane_entry<R>(C->sinl, l);
  }
  const R m00 = sum8(p0), m01 = sum8(p1 * cl), m02 = sum8(p1 * sl);
  const R m11 = sum8(p2 * cl * cl), m12 = sum8(p2 * cl * sl), m22 = sum8(p2 * sl * sl);
  if (l == 0) {
    s_mom[0][ts] = (double)m00;
    s_mom[1][ts] = (double)m01;
    s_mom[2][ts] = (double)m02;
    s_mom[3][ts] = (double)m11;
    s_mom[4][ts] = (double)m12;
    s_mom[5][ts] = (double)m22;
    s_mom[6][ts] = lnM;
  }
  if constexpr (kMu) {  // the particle current for the n matching
    R c0, c1;
    slice_current(f, C, &c0, &c1);
    const R n0 = sum8(c0), n1 = sum8(c1 * cl), n2 = sum8(c1 * sl);
    if (l == 0) {
      s_mom[7][ts] = (double)n0;
      s_mom[8][ts] = (double)n1;
      s_mom[9][ts] = (double)n2;
    }
  }
}
// Matching and record of site (sx, sy) of the tile from the sums in LDS
// column t.
template <typename R, int kTY, int kMu>
__device__ __forceinline__ void match_site(int t, int sx, int sy, const EosTable* __restrict__ tbg,
                                           const StageArgs& a, double* __restrict__ sc, int* __restrict__ err,
                                           double (*s_mom)[kTX * kTY]) {
  const int ss = sy * a.nx + sx;
  const double lnMs = s_mom[6][t];
  // The mixed tensor T_kin g = G (sum w F V V) g with G = M^4/(2 pi^2): its
  // timelike eigenvector does not depend on G, and its eigenvalue is
  // lambda = G lambda', so the matching runs on the sums themselves and
  // ln lambda = ln lambda' + 4 ln M - ln(2 pi^2) (no exp of ln M in FP64)
  double tk[6];
  bool finite = true;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    tk[i] = s_mom[i][t];
    finite = finite && isfinite(tk[i]);
  }
  finite = finite && isfinite(lnMs);
  double lamp, u[3];
  const bool matched = landau3(tk, &lamp, u);
  const double ln2pi2 = 2.9826069522587457;  // ln(2 pi^2)
  const double glam = log(lamp) + 4.0 * lnMs - ln2pi2;
  EosAt E;
  const EosTable tb = load_table(tbg);  // read here, where it is used
  bool eos_ok;
  double alpha = 0.0;
  double M;
  if constexpr (kMu) {
    M = exp(lnMs);
    const double G = M * M * M * M * (1.0 / (2.0 * kPi * kPi));
    // n = u_a N^a with N^a = M^3/(2 pi^2) sum w F V^a (eq. (NTdisc))
    const double n = G / M * (u[0] * s_mom[7][t] - u[1] * s_mom[8][t] - u[2] * s_mom[9][t]);
    eos_ok = eos_mu(tb, G * lamp, n, &E, &alpha);
  } else {
    // the record holds M in the node precision: FP32 needs no FP64 exp
    M = sizeof(R) == 4 ? (double)__expf((float)lnMs) : exp(lnMs);
    eos_ok = eos_g(tb, glam, lamp > 0.0, &E);
  }
  if (!finite) flag(err, kErrNonfinite);
  else if (!matched) flag(err, kErrMatch);
  else if (!eos_ok) flag(err, kErrEos);
  const double invT = 1.0 / E.T;
  SiteRecord<R> rec;
  rec.v[kScUt] = (R)u[0];
  rec.v[kScUx] = (R)u[1];
  rec.v[kScUy] = (R)u[2];
  rec.v[kScM] = (R)M;
  rec.v[kScMeq] = (R)E.M_eq;
  rec.v[kScRate] = (R)(E.T * a.inv_eta_hbarc / E.q);  // 1/tau_R [fm^-1]
  rec.v[kScMinvT] = (R)(M * invT);
  rec.v[kScL2invT] = (R)(1.4426950408889634 * invT);  // log2(e)/T
  rec.beta = kMu ? alpha : E.beta;  // beta = 0 for the constant mass of the mu mode
  rec.lnM = lnMs;
  store_record<R>(buf_rsrc(sc, (uint32_t)a.n_sites * SiteRecord<R>::kBytes), ss, rec);
}
// The block's barrier, then threads 0 .. 8 kTY - 1 match one site each.
template <typename R, int kTY, int kMu>
__device__ __forceinline__ void match_sites(int t, int bx, int by, const EosTable* __restrict__ tbg,
                                            const StageArgs& a, double* __restrict__ sc, int* __restrict__ err,
                                            double (*s_mom)[kTX * kTY]) {
  constexpr int kTile = kTX * kTY;
  __syncthreads();
  const int sx = bx * kTX + (t % kTX), sy = by * kTY + (t / kTX);
  if (t < kTile && sx < a.nx && sy < a.ny) match_site<R, kTY, kMu>(t, sx, sy, tbg, a, sc, err, s_mom);
}

// Tile of a block in the XCD-aware order: workgroups go round-robin over the
// eight XCDs, so XCD (blockIdx % 8) is given the contiguous band of
// row-major tiles [xcd * per, (xcd + 1) * per) and sweeps it in dispatch
// order; the x and y neighbours of a tile then sit in the same L2.
__device__ __forceinline__ int xcd_tile(int n_tiles) {
  const int per = (n_tiles + kXcds - 1) / kXcds;
  return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// Geometry of one lane in a tile: site (x, y) (site 0 for lanes outside the
// grid, which compute but store nothing) and its byte offset in a plane.
struct LaneSite {
  int bx, by, x, y, site;
  bool valid;
  uint32_t me;
};
template <typename R, int kTY>
__device__ __forceinline__ LaneSite lane_site(int tile, int tiles_x, int ts, int l, const StageArgs& a) {
  LaneSite g;
  g.bx = tile % tiles_x;
  g.by = tile / tiles_x;
  const int x0 = g.bx * kTX + (ts % kTX), y0 = g.by * kTY + (ts / kTX);
  g.valid = (x0 < a.nx) && (y0 < a.ny);
  g.x = g.valid ? x0 : 0;
  g.y = g.valid ? y0 : 0;
  g.site = g.y * a.nx + g.x;
  g.me = ((uint32_t)g.site * kSl + l) * (uint32_t)sizeof(R);
  return g;
}


// Stage kernel of one event: one block per 8 x kTY tile, blocks in the
// XCD-aware tile order of xcd_tile.  kStream = kNT streams the new state
// past the caches (stores, and the corrector's base slice, read once) for
// states larger than the last-level cache; 0 keeps them cached.
template <typename R, int STAGE, int kTY = TileRows<R>::v, int kStream = 0, int kForce = 0, int kMu = 0,
          int kGrad = 0>
__global__ __launch_bounds__(kTX * kTY * kSl, (kForce ? ForceWaves<R>::v : (kMu ? MuWaves<R>::v : MinWaves<R, STAGE>::v))) void stage_kernel(
    const R* __restrict__ Fin, const R* __restrict__ Fbase, R* __restrict__ Fout,
    const double* __restrict__ lnMin, const double* __restrict__ lnMbase, double* __restrict__ lnMout,
    const double* __restrict__ scin, double* __restrict__ scout, const StageConst<R>* __restrict__ Cg,
    const EosTable* __restrict__ tbg, const StageArgs a, int* __restrict__ err) {
  __shared__ double s_mom[kMomRows][kTX * kTY];
  // exchange area of the 3-D force: per wave 25 nodes x 64 lanes
  __shared__ __attribute__((aligned(16))) R s_force[kForce ? kTY * 25 * 64 : 1];
  const int n_tiles = ((a.nx + kTX - 1) / kTX) * ((a.ny + kTY - 1) / kTY);
  const int tile = xcd_tile(n_tiles);
  if (tile >= n_tiles) return;  // whole block
#include "stage_body.inc"
}

// Batched stage: the launch's tiles are the tiles of all events in turn
// (event e owns tiles [tile0_e, tile0_e + tiles_e)), taken in the XCD-aware
// order; each block looks up its event and runs the single-event tile code,
// so an event's result does not depend on the batch it is in.
template <typename R, int STAGE, int kTY, int kW, int kStream, int kForce, int kMu, int kGrad>
__global__ __launch_bounds__(kTX * kTY * kSl, kW) void batch_stage_kernel(
    const BatchEvent* __restrict__ ev, const int32_t* __restrict__ tile_event, int n_tiles, StageTime time,
    const StageTime* __restrict__ times, int time_idx, int i_in, int i_base, int i_out,
    const StageConst<R>* __restrict__ Cg, const EosTable* __restrict__ tbg, StageArgs a,
    int* __restrict__ err) {
  __shared__ double s_mom[kMomRows][kTX * kTY];
  __shared__ __attribute__((aligned(16))) R s_force[kForce ? kTY * 25 * 64 : 1];
  const int tile = xcd_tile(n_tiles);
  if (tile >= n_tiles) return;  // whole block
  // the event, its buffers and the stage time through constant-address
  // pointers: uniform values, read with scalar loads
  typedef const __attribute__((address_space(4))) BatchEvent* EvP;
  typedef const __attribute__((address_space(4))) int32_t* TeP;
  typedef const __attribute__((address_space(4))) StageTime* TmP;
  const int e = ((TeP)(uint64_t)tile_event)[tile];
  const EvP ep = (EvP)(uint64_t)ev + e;
  struct {
    int32_t tile0;
  } E;
  E.tile0 = ep->tile0;
  if (times) {
    const TmP tp = (TmP)(uint64_t)times + time_idx;
    time.tau = tp->tau;
    time.tau_s = tp->tau_s;
    time.inv_tau_s = tp->inv_tau_s;
  }
  a.nx = ep->nx;
  a.ny = ep->ny;
  a.n_sites = ep->n_sites;
  a.inv2dx = ep->inv2dx;
  a.inv_dx = 2.0 * a.inv2dx;
  a.inv_eta_hbarc = ep->inv_eta_hbarc;
  a.tau = time.tau;
  a.tau_s = time.tau_s;
  a.inv_tau_s = time.inv_tau_s;
  // only the buffers this stage touches (scalar loads at uniform offsets)
  const R* __restrict__ Fin = (const R*)ep->F[i_in];
  const R* __restrict__ Fbase = (const R*)ep->F[i_base];
  R* __restrict__ Fout = (R*)ep->F[i_out];
  const double* __restrict__ lnMin = ep->lnM[i_in];
  const double* __restrict__ lnMbase = ep->lnM[i_base];
  double* __restrict__ lnMout = ep->lnM[i_out];
  const double* __restrict__ scin = ep->sc[i_in];
  double* __restrict__ scout = ep->sc[i_out];
  {
    const int tile_g = tile;
    {
      const int tile = tile_g - E.tile0;  // within the event
#include "stage_body.inc"
    }
  }
}

// Site scalars of a state that no stage produced (after lb_init or
// lb_set_state): the matching phase of the stage kernel on its own.
template <typename R, int kMu>
__global__ __launch_bounds__(kTX * TileRows<R>::v * kSl) void site_kernel(
    const R* __restrict__ F, const double* __restrict__ lnMv, double* __restrict__ sc,
    const StageConst<R>* __restrict__ Cg, const EosTable* __restrict__ tbg, const StageArgs a,
    int* __restrict__ err) {
  const CPtr<R> C = const_ptr(Cg);
  constexpr int kTY = TileRows<R>::v;
  __shared__ double s_mom[kMomRows][kTX * kTY];
  const int t = threadIdx.x;
  const int ts = t >> 3, l = t & 7;
  const int tiles_x = (a.nx + kTX - 1) / kTX;
  const int n_tiles = tiles_x * ((a.ny + kTY - 1) / kTY);
  const int tile = xcd_tile(n_tiles);
  if (tile >= n_tiles) return;
  const int bx = tile % tiles_x, by = tile / tiles_x;
  const int x0 = bx * kTX + (ts % kTX), y0 = by * kTY + (ts / kTX);
  const bool valid = (x0 < a.nx) && (y0 < a.ny);
  const int site = valid ? y0 * a.nx + x0 : 0;
  const R cl = lane_load<R>(C->cosl, l), sl = lane_load<R>(C->sinl, l);
  R f[25];
  load_slice<R>(buf_rsrc(F, (uint32_t)a.n_sites * kSl * 25u * (uint32_t)sizeof(R)), (uint32_t)site * kSl + l,
                NodeLayout<R>::gbytes(a.n_sites), f);
  match_moments<R, kTY, kMu>(f, C, cl, sl, lnMv[site], t, s_mom);
  match_sites<R, kTY, kMu>(t, bx, by, tbg, a, sc, err, s_mom);
}

// Initial local equilibrium (Sec. IV.D): T0 from eps_EoS(T0) = e0.
template <typename R, int NXI, int NTH>
__global__ __launch_bounds__(kBlock) void init_kernel(const double* __restrict__ e0,
                                                      const double* __restrict__ ux0,
                                                      const double* __restrict__ uy0, R* __restrict__ F,
                                                      double* __restrict__ lnM,
                                                      const LatticeConst<R, NXI, NTH> C,
                                                      const EosTable tb, const StageArgs a,
                                                      int* __restrict__ err) {
  constexpr int Q = NXI * NTH;
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  const int site = tid >> 3;
  const int l = tid & 7;
  if (site >= a.n_sites) return;
  // with mu0 = alpha0 T0 (constant mass): eps0(T0) = e0 exp(-alpha0)
  const double e = e0[site] * (kHbarC * kHbarC * kHbarC) * exp(-a.alpha0);
  const double vx = ux0 ? ux0[site] : 0.0, vy = uy0 ? uy0[site] : 0.0;
  int bad = 0;
  if (!isfinite(e) || !(e > 0.0) || !isfinite(vx) || !isfinite(vy)) bad = kErrNonfinite;
  double uu = tb.u_lo;
  if (!bad && !eos_invert(tb, kLnEeos, tb.inv_ee, tb.ge0, tb.ge_h, tb.ge_inv_h, log(e), &uu)) bad = kErrEos;
  if (!bad && (uu < tb.u_lo || uu > tb.u_hi)) bad = kErrEos;
  if (bad) uu = tb.u_lo;
  double t, w[4], dw[4];
  const int i = eos_locate(tb, uu, &t);
  lagrange4(t, w, dw);
  const double T0 = exp(uu);
  const double M = eos_field(tb, i, w, kZ) * T0;
  const double ut = sqrt(1.0 + vx * vx + vy * vy);
  const double cu = vx * (double)C.cosl[l] + vy * (double)C.sinl[l];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = q / NTH;
    const double uP = M * (ut * (double)C.x[k] - cu * (double)C.sig[q]);
    F[NodeLayout<R>::offset(q, site, l, a.n_sites) / sizeof(R)] = (R)(a.Z * exp(a.alpha0 - uP / T0));
  }
  if (l == 0) {
    lnM[site] = log(M);
    if (bad) flag(err, bad);
  }
}

// ---------------------------------------------------------------------------
// Observables: T^{ab} with B g^{ab}, N^a, T, u, M (eqs. (emtnew), (NTdisc)).
template <typename R, int NXI, int NTH>
__global__ __launch_bounds__(kBlock) void moments_kernel(const R* __restrict__ F,
                                                         const double* __restrict__ lnMv,
                                                         double* __restrict__ out,
                                                         const LatticeConst<R, NXI, NTH> C,
                                                         const EosTable tb, const StageArgs a,
                                                         int* __restrict__ err) {
  constexpr int Q = NXI * NTH;
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  const int site = tid >> 3;
  const int l = tid & 7;
  if (site >= a.n_sites) return;
  double p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0, p5 = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double fq = (double)F[NodeLayout<R>::offset(q, site, l, a.n_sites) / sizeof(R)];
    p0 += (double)C.wx2[q] * fq;
    p1 += (double)C.wxs[q] * fq;
    p2 += (double)C.ws2[q] * fq;
    p3 += (double)C.wvY2[q] * fq;
    p4 += (double)C.wx[q] * fq;
    p5 += (double)C.w[q] * (double)C.sig[q] * fq;
  }
  const double cl = (double)C.cosl[l], sl = (double)C.sinl[l];
  const double m00 = sum8(p0), m01 = sum8(p1 * cl), m02 = sum8(p1 * sl);
  const double m11 = sum8(p2 * cl * cl), m12 = sum8(p2 * cl * sl), m22 = sum8(p2 * sl * sl);
  const double mYY = sum8(p3), n0 = sum8(p4), n1 = sum8(p5 * cl), n2 = sum8(p5 * sl);
  const double lnM = lnMv[site];
  const double M = exp(lnM);
  const double G = M * M * M * M / (2.0 * kPi * kPi);
  const double G3 = M * M * M / (2.0 * kPi * kPi);
  const double tk[6] = {G * m00, G * m01, G * m02, G * m11, G * m12, G * m22};
  double lam, u[3];
  const bool matched = landau3(tk, &lam, u);
  EosAt E;
  double alpha;
  const bool eos_ok = a.mu_mode ? eos_mu(tb, lam, G3 * (u[0] * n0 - u[1] * n1 - u[2] * n2), &E, &alpha)
                                : eos_from_lambda(tb, lam, &E);
  if (l == 0) {
    bool finite = true;
    for (int i = 0; i < 6; ++i) finite = finite && isfinite(tk[i]);
    if (!finite) flag(err, kErrNonfinite);
    else if (!matched) flag(err, kErrMatch);
    else if (!eos_ok) flag(err, kErrEos);
    const double B = E.Bt4 * E.T * E.T * E.T * E.T;
    const double c3 = 1.0 / (kHbarC * kHbarC * kHbarC);
    const size_t ns = (size_t)a.n_sites;
    out[0 * ns + site] = (tk[0] + B) * c3;
    out[1 * ns + site] = tk[1] * c3;
    out[2 * ns + site] = tk[2] * c3;
    out[3 * ns + site] = (tk[3] - B) * c3;
    out[4 * ns + site] = tk[4] * c3;
    out[5 * ns + site] = (tk[5] - B) * c3;
    out[6 * ns + site] = (G * mYY - B) * c3;
    out[7 * ns + site] = G3 * n0 * c3;
    out[8 * ns + site] = G3 * n1 * c3;
    out[9 * ns + site] = G3 * n2 * c3;
    out[10 * ns + site] = E.T;
    out[11 * ns + site] = u[1];
    out[12 * ns + site] = u[2];
    out[13 * ns + site] = M;
  }
}

// ---------------------------------------------------------------------------
template <typename R>
__global__ void get_state_kernel(const R* __restrict__ F, double* __restrict__ Fc, int n_q, int n_sites) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)n_q * n_sites * kSl;
  if (i >= total) return;
  // thread i = (q * n_sites + site) * 8 + l
  const int l = (int)(i % kSl);
  const size_t rest = i / kSl;
  const int site = (int)(rest % n_sites);
  const int q = (int)(rest / n_sites);
  Fc[((size_t)q * kSl + l) * n_sites + site] = (double)F[NodeLayout<R>::offset(q, site, l, n_sites) / sizeof(R)];
}

template <typename R>
__global__ void set_state_kernel(const double* __restrict__ Fc, R* __restrict__ F, int n_q, int n_sites) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)n_q * n_sites * kSl;
  if (i >= total) return;
  const int l = (int)(i % kSl);
  const size_t rest = i / kSl;
  const int site = (int)(rest % n_sites);
  const int q = (int)(rest / n_sites);
  F[NodeLayout<R>::offset(q, site, l, n_sites) / sizeof(R)] = (R)Fc[((size_t)q * kSl + l) * n_sites + site];
}

// ---------------------------------------------------------------------------
namespace {
inline dim3 grid_for(int n_sites) { return dim3((unsigned)(((size_t)n_sites * kSl + kBlock - 1) / kBlock)); }
}  // namespace

namespace {
// one stage of the single-event kernel with the given template flags
template <typename R, int kTY, int kStream, int kForce, int kMu, int kGrad = 0>
hipError_t stage_launch_t(int stage, dim3 g, dim3 b, const void* Fin, const void* Fbase, void* Fout,
                          const double* lnMin, const double* lnMbase, double* lnMout, const double* scin,
                          double* scout, const void* sc, const EosTable* tb, const StageArgs& a, int* err,
                          hipStream_t s) {
  const auto* C = static_cast<const StageConst<R>*>(sc);
  if (stage == 0)
    hipLaunchKernelGGL((stage_kernel<R, 0, kTY, kStream, kForce, kMu, kGrad>), g, b, 0, s, (const R*)Fin,
                       (const R*)Fbase, (R*)Fout, lnMin, lnMbase, lnMout, scin, scout, C, tb, a, err);
  else
    hipLaunchKernelGGL((stage_kernel<R, 1, kTY, kStream, kForce, kMu, kGrad>), g, b, 0, s, (const R*)Fin,
                       (const R*)Fbase, (R*)Fout, lnMin, lnMbase, lnMout, scin, scout, C, tb, a, err);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_force_columns(const void* cst64, double* G, hipStream_t s) {
  hipLaunchKernelGGL(force_columns_kernel, dim3(25, 2), dim3(64), 0, s,
                     static_cast<const StageConst<double>*>(cst64), G);
  return hipGetLastError();
}

hipError_t launch_stage(int precision, int stage, const void* Fin, const void* Fbase, void* Fout,
                        const double* lnMin, const double* lnMbase, double* lnMout, const double* scin,
                        double* scout, const void* sc, const EosTable* tb, const StageArgs& a, int* err,
                        hipStream_t s) {
  // FP32 states whose three buffers exceed the last-level cache: 8-row
  // tiles and streaming stores (measured 5-6% faster per step at 512 x 512,
  // 20% slower at 256 x 256, where the state stays in the cache); the
  // weak-form 3-D force and the conserved particle number run with the
  // default tiles and cached stores
  const bool force3d = a.force_form == LB_FORCE_WEAK3D, mu = a.mu_mode != 0;
  const bool upwind = a.grad_form == LB_GRAD_UPWIND;  // force on F_eq only (host check)
  const bool big = !force3d && !mu && precision == LB_FP32_FP64MATCH &&
                   (size_t)a.n_sites * kSl * 25 * sizeof(float) * 3 > kMallBytes;
  const int ty = precision == LB_FP32_FP64MATCH ? (big ? kBigTileRows : TileRows<float>::v) : TileRows<double>::v;
  const unsigned tiles = (unsigned)(((a.nx + kTX - 1) / kTX) * ((a.ny + ty - 1) / ty));
  const unsigned per = (tiles + kXcds - 1) / kXcds;
  const dim3 g(per * kXcds), b(kTX * ty * kSl);
#define LB_STAGE_ARGS stage, g, b, Fin, Fbase, Fout, lnMin, lnMbase, lnMout, scin, scout, sc, tb, a, err, s
  if (precision == LB_FP32_FP64MATCH) {
    constexpr int TY = TileRows<float>::v;
    if (big) return upwind ? stage_launch_t<float, kBigTileRows, kNT, 0, 0, 1>(LB_STAGE_ARGS)
                           : stage_launch_t<float, kBigTileRows, kNT, 0, 0>(LB_STAGE_ARGS);
    if (upwind)
      return mu ? stage_launch_t<float, TY, 0, 0, 1, 1>(LB_STAGE_ARGS) : stage_launch_t<float, TY, 0, 0, 0, 1>(LB_STAGE_ARGS);
    if (force3d)
      return mu ? stage_launch_t<float, TY, 0, 1, 1>(LB_STAGE_ARGS) : stage_launch_t<float, TY, 0, 1, 0>(LB_STAGE_ARGS);
    return mu ? stage_launch_t<float, TY, 0, 0, 1>(LB_STAGE_ARGS) : stage_launch_t<float, TY, 0, 0, 0>(LB_STAGE_ARGS);
  }
  constexpr int TY = TileRows<double>::v;
  if (upwind)
    return mu ? stage_launch_t<double, TY, 0, 0, 1, 1>(LB_STAGE_ARGS) : stage_launch_t<double, TY, 0, 0, 0, 1>(LB_STAGE_ARGS);
  if (force3d)
    return mu ? stage_launch_t<double, TY, 0, 1, 1>(LB_STAGE_ARGS) : stage_launch_t<double, TY, 0, 1, 0>(LB_STAGE_ARGS);
  return mu ? stage_launch_t<double, TY, 0, 0, 1>(LB_STAGE_ARGS) : stage_launch_t<double, TY, 0, 0, 0>(LB_STAGE_ARGS);
#undef LB_STAGE_ARGS
}

namespace {
template <typename R, int STAGE, int kTY, int kW, int kStream, int kForce = 0, int kMu = 0, int kGrad = 0>
hipError_t batch_launch_t(const BatchEvent* ev, const int32_t* te, int n_tiles, StageTime time,
                          const StageTime* times, int tidx, int i_in, int i_base, int i_out, const void* sc,
                          const EosTable* tb, const StageArgs& a, int* err, hipStream_t s) {
  const unsigned per = (unsigned)((n_tiles + kXcds - 1) / kXcds);
  hipLaunchKernelGGL((batch_stage_kernel<R, STAGE, kTY, kW, kStream, kForce, kMu, kGrad>), dim3(per * kXcds), dim3(kTX * kTY * kSl), 0, s, ev,
                     te, n_tiles, time, times, tidx, i_in, i_base, i_out, static_cast<const StageConst<R>*>(sc), tb,
                     a, err);
  return hipGetLastError();
}
// variant v of the batched kernel: tile rows kBatchTileRows[v % 3]; FP32
// (v / 3) % 2 = 0: 4 waves per SIMD, 1: 3, and v >= 6 streaming stores;
// FP64: 2 waves per SIMD
template <typename R, int STAGE>
hipError_t batch_launch_s(int variant, const BatchEvent* ev, const int32_t* te, int n_tiles, StageTime time,
                          const StageTime* times, int tidx, int i_in, int i_base, int i_out, const void* sc,
                          const EosTable* tb, const StageArgs& a, int* err, hipStream_t s) {
#define LB_BATCH_CASE(V, TY, W, NT)                                                                               \
  case V:                                                                                                        \
    return batch_launch_t<R, STAGE, TY, W, NT>(ev, te, n_tiles, time, times, tidx, i_in, i_base, i_out, sc, tb, a,  \
                                               err, s);
#define LB_BATCH_CASE_FM(V, TY, W, F, MU)                                                                         \
  case V:                                                                                                        \
    return batch_launch_t<R, STAGE, TY, W, 0, F, MU>(ev, te, n_tiles, time, times, tidx, i_in, i_base, i_out, sc,  \
                                                     tb, a, err, s);
#define LB_BATCH_CASE_UP(V, TY, W, MU)                                                                            \
  case V:                                                                                                        \
    return batch_launch_t<R, STAGE, TY, W, 0, 0, MU, 1>(ev, te, n_tiles, time, times, tidx, i_in, i_base, i_out, \
                                                        sc, tb, a, err, s);
  // the weak-form 3-D force and/or the conserved particle number: tile rows
  // 2, 4, 8 at the occupancy of the single-event kernel (a block of 8 rows
  // is 8 waves, so at least 2 waves per SIMD); both together at the
  // force's occupancy, as lb_step runs them
  // the upwind ln M gradient (force on F_eq; with or without the conserved
  // particle number): tile rows 2, 4, 8 at the default kernels' occupancy
  if (a.grad_form == LB_GRAD_UPWIND) {
    constexpr int W = sizeof(R) == 8 ? 2 : 4;
    if (a.mu_mode) {
      switch (variant) {
        LB_BATCH_CASE_UP(0, 2, MuWaves<R>::v, 1)
        LB_BATCH_CASE_UP(1, 4, MuWaves<R>::v, 1)
        LB_BATCH_CASE_UP(2, 8, MuWaves<R>::v, 1)
        default: return hipErrorInvalidValue;
      }
    }
    switch (variant) {
      LB_BATCH_CASE_UP(0, 2, W, 0)
      LB_BATCH_CASE_UP(1, 4, W, 0)
      LB_BATCH_CASE_UP(2, 8, W, 0)
      default: return hipErrorInvalidValue;
    }
  }
  if (a.force_form == LB_FORCE_WEAK3D && a.mu_mode) {
    switch (variant) {
      LB_BATCH_CASE_FM(0, 2, ForceWaves<R>::v, 1, 1)
      LB_BATCH_CASE_FM(1, 4, ForceWaves<R>::v, 1, 1)
      LB_BATCH_CASE_FM(2, 8, 2, 1, 1)
      default: return hipErrorInvalidValue;
    }
  }
  if (a.force_form == LB_FORCE_WEAK3D) {
    switch (variant) {
      LB_BATCH_CASE_FM(0, 2, ForceWaves<R>::v, 1, 0)
      LB_BATCH_CASE_FM(1, 4, ForceWaves<R>::v, 1, 0)
      LB_BATCH_CASE_FM(2, 8, 2, 1, 0)
      default: return hipErrorInvalidValue;
    }
  }
  if (a.mu_mode) {
    switch (variant) {
      LB_BATCH_CASE_FM(0, 2, MuWaves<R>::v, 0, 1)
      LB_BATCH_CASE_FM(1, 4, MuWaves<R>::v, 0, 1)
      LB_BATCH_CASE_FM(2, 8, MuWaves<R>::v, 0, 1)
      default: return hipErrorInvalidValue;
    }
  }
  if constexpr (sizeof(R) == 8) {
    switch (variant) {
      LB_BATCH_CASE(0, 2, 2, 0)
      LB_BATCH_CASE(1, 4, 2, 0)
      LB_BATCH_CASE(2, 8, 2, 0)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (variant) {
      LB_BATCH_CASE(0, 2, 4, 0)
      LB_BATCH_CASE(1, 4, 4, 0)
      LB_BATCH_CASE(2, 8, 4, 0)
      LB_BATCH_CASE(3, 2, 3, 0)
      LB_BATCH_CASE(4, 4, 3, 0)
      LB_BATCH_CASE(5, 8, 3, 0)
      LB_BATCH_CASE(6, 2, 4, kNT)
      LB_BATCH_CASE(7, 4, 4, kNT)
      LB_BATCH_CASE(8, 8, 4, kNT)
      LB_BATCH_CASE(9, 2, 3, kNT)
      LB_BATCH_CASE(10, 4, 3, kNT)
      LB_BATCH_CASE(11, 8, 3, kNT)
      default: return hipErrorInvalidValue;
    }
  }
#undef LB_BATCH_CASE
#undef LB_BATCH_CASE_FM
#undef LB_BATCH_CASE_UP
}
}  // namespace

hipError_t launch_batch_stage(int precision, int stage, int variant, const BatchEvent* ev,
                              const int32_t* tile_event, int n_tiles, StageTime time, const StageTime* times,
                              int time_idx, int i_in, int i_base, int i_out, const void* sc, const EosTable* tb,
                              const StageArgs& a, int* err, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (precision == LB_FP32_FP64MATCH)
    return stage == 0 ? batch_launch_s<float, 0>(variant, ev, tile_event, n_tiles, time, times, time_idx, i_in,
                                                 i_base, i_out, sc, tb, a, err, s)
                      : batch_launch_s<float, 1>(variant, ev, tile_event, n_tiles, time, times, time_idx, i_in,
                                                 i_base, i_out, sc, tb, a, err, s);
  return stage == 0 ? batch_launch_s<double, 0>(variant, ev, tile_event, n_tiles, time, times, time_idx, i_in,
                                                i_base, i_out, sc, tb, a, err, s)
                    : batch_launch_s<double, 1>(variant, ev, tile_event, n_tiles, time, times, time_idx, i_in,
                                                i_base, i_out, sc, tb, a, err, s);
}

hipError_t launch_site(int precision, const void* F, const double* lnM, double* scout, const void* sc,
                       const EosTable* tb, const StageArgs& a, int* err, hipStream_t s) {
  const int ty = precision == LB_FP32_FP64MATCH ? TileRows<float>::v : TileRows<double>::v;
  const unsigned tiles = (unsigned)(((a.nx + kTX - 1) / kTX) * ((a.ny + ty - 1) / ty));
  const unsigned per = (tiles + kXcds - 1) / kXcds;
  const dim3 g(per * kXcds), b(kTX * ty * kSl);
  if (precision == LB_FP32_FP64MATCH) {
    const auto* C = static_cast<const StageConst<float>*>(sc);
    if (a.mu_mode)
      hipLaunchKernelGGL((site_kernel<float, 1>), g, b, 0, s, (const float*)F, lnM, scout, C, tb, a, err);
    else
      hipLaunchKernelGGL((site_kernel<float, 0>), g, b, 0, s, (const float*)F, lnM, scout, C, tb, a, err);
  } else {
    const auto* C = static_cast<const StageConst<double>*>(sc);
    if (a.mu_mode)
      hipLaunchKernelGGL((site_kernel<double, 1>), g, b, 0, s, (const double*)F, lnM, scout, C, tb, a, err);
    else
      hipLaunchKernelGGL((site_kernel<double, 0>), g, b, 0, s, (const double*)F, lnM, scout, C, tb, a, err);
  }
  return hipGetLastError();
}

hipError_t launch_init(int precision, const double* e0, const double* ux0, const double* uy0, void* F,
                       double* lnM, const void* lc, const EosTable& tb, const StageArgs& a, int* err,
                       hipStream_t s) {
  const dim3 g = grid_for(a.n_sites), b(kBlock);
  if (precision == LB_FP32_FP64MATCH)
    hipLaunchKernelGGL((init_kernel<float, 5, 5>), g, b, 0, s, e0, ux0, uy0, (float*)F, lnM,
                       *static_cast<const LatticeConst<float, 5, 5>*>(lc), tb, a, err);
  else
    hipLaunchKernelGGL((init_kernel<double, 5, 5>), g, b, 0, s, e0, ux0, uy0, (double*)F, lnM,
                       *static_cast<const LatticeConst<double, 5, 5>*>(lc), tb, a, err);
  return hipGetLastError();
}

hipError_t launch_moments(int precision, const void* F, const double* lnM, double* out, const void* lc,
                          const EosTable& tb, const StageArgs& a, int* err, hipStream_t s) {
  const dim3 g = grid_for(a.n_sites), b(kBlock);
  if (precision == LB_FP32_FP64MATCH)
    hipLaunchKernelGGL((moments_kernel<float, 5, 5>), g, b, 0, s, (const float*)F, lnM, out,
                       *static_cast<const LatticeConst<float, 5, 5>*>(lc), tb, a, err);
  else
    hipLaunchKernelGGL((moments_kernel<double, 5, 5>), g, b, 0, s, (const double*)F, lnM, out,
                       *static_cast<const LatticeConst<double, 5, 5>*>(lc), tb, a, err);
  return hipGetLastError();
}

hipError_t launch_get_state(int precision, const void* F, double* Fc, int n_q, int n_sites, hipStream_t s) {
  const size_t total = (size_t)n_q * n_sites * kSl;
  const dim3 g((unsigned)((total + 255) / 256)), b(256);
  if (precision == LB_FP32_FP64MATCH)
    hipLaunchKernelGGL(get_state_kernel<float>, g, b, 0, s, (const float*)F, Fc, n_q, n_sites);
  else
    hipLaunchKernelGGL(get_state_kernel<double>, g, b, 0, s, (const double*)F, Fc, n_q, n_sites);
  return hipGetLastError();
}

hipError_t launch_set_state(int precision, const double* Fc, void* F, int n_q, int n_sites, hipStream_t s) {
  const size_t total = (size_t)n_q * n_sites * kSl;
  const dim3 g((unsigned)((total + 255) / 256)), b(256);
  if (precision == LB_FP32_FP64MATCH)
    hipLaunchKernelGGL(set_state_kernel<float>, g, b, 0, s, Fc, (float*)F, n_q, n_sites);
  else
    hipLaunchKernelGGL(set_state_kernel<double>, g, b, 0, s, Fc, (double*)F, n_q, n_sites);
  return hipGetLastError();
}

}  // namespace lbmi
