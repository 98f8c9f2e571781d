// Internal host/device data layouts of the lensfield library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lf {

// Member galaxies are stored sorted into profile segments so that every halo loop
// in a kernel is uniform (one closed form per loop, no per-halo branching).
enum Seg { SEG_CPJE = 0, SEG_EPJE, SEG_CSIE, SEG_ESIE, SEG_POINT, SEG_NFW, SEG_ENFW, NSEG };

struct Bind {            // mirrors lf_binding
  int32_t kind, index, xf, pad;
  double value;
};
struct MainDesc {        // mirrors lf_component
  int32_t type, pad;
  Bind f[7];             // x, y, b, q, pa, s, a
};

// Constants that turn raw bound values into lensing units at the model's lens redshift.
struct XfConst {
  double arcsec_per_kpc;  // 1 kpc at D_d in arcsec
  double rho_c;           // critical density at z_d [Msun / Mpc^3]
  double sigma_cr;        // a_dis-free critical surface density c^2/(4 pi G D_d) [Msun / Mpc^2]
  double Dd;              // D(0, z_d) [Mpc]
};

// Per-(sample, main component) record, FP64, produced by the expansion kernel.
struct MainRec {
  double x, y, b, q, c, sn, s, a;   // c, sn = cos, sin of the position angle
  double e, bqe, q2, pad;           // e = sqrt(1 - q^2), bqe = b q / e, q2 = q^2
  int32_t type, flags, pad0, pad1;
};

// Member catalog entry, fixed across samples: factors multiplied by per-sample scalars.
struct MemCat {
  double x, y, fb, fs, fa, q, c, sn;
};

// FP32 copy of the member catalog for the per-lane scaled chi^2 path.  The centre is kept
// as an unevaluated FP32 pair (x = xh + xl to 48 bits) so that a point-centre offset can be
// formed in FP32 with a relative error of a few ulp whatever the absolute coordinates.
struct MemCat32 {
  float xh, xl, yh, yl;
  float fb, fs, fa, q, c, sn, fbk2, pad1;   // fbk2 = (NEAR_K fb / q)^2
};

// Per-sample member multipliers (b*, s*, a*) and sample validity flags.
struct MulRec {
  double b, s, a;
  int32_t flags, pad;
};

// Near field of the FP32 member path: a member's term at a point closer than
// NEAR_K * b / q (where the term's deformation exceeds about 1/NEAR_K, so FP32 rounding of the
// term alone would exceed ~1e-7) is evaluated from the FP64 record instead.
static constexpr double NEAR_K = 3.0;

// Pre-scaled member record for one sample.  The FP32 flavour keeps the centre as an FP32
// pair (as in MemCat32).  bd = b (a - s) and apls = a + s are formed in FP64 before rounding
// (they feed the cancellation-free dPIE form); rn2 is the squared near-field radius.
// fm, fw: coefficients of the far-field expansion of a circular dPIE in t = 1/r (valid for
// r >= FAR_K a): m = u (fm0 + t (fm1 + u (fm2 + u (fm3 + u (fm4 + u fm5))))) and
// w = u^2 (fw0 + t (fw1 + u (...))), u = t^2 (see lf_segs.h).  The coefficients of
// w' = dw/d(r^2) = u^3 (fwp0 + t (fwp1 + u (...))) are fixed multiples of fm (FAR_WP) and are
// formed when a record is staged for third derivatives.
struct MemRec32 {
  float xh, xl, yh, yl;
  float b, s, a, s2, a2, bd, apls, rn2;   // the circular segments read these 12 words only
  float c, sn, q2, e, bqe, pad0, pad1, pad2;
  float fm[6], fw[6];
};

// Far field of a circular dPIE member: at r >= FAR_K a the truncated expansion of its closed
// form in 1/r (terms through 1/r^11) is exact to 4e-9 (m) and 3e-8 (w) relative, below FP32
// rounding; farther out fewer terms reach the same bound: five (through 1/r^9) at r >= FAR_K5 a
// (6e-9, 4e-8) and four (through 1/r^7) at r >= FAR_K4 a (5e-9, 2e-8), for cores s <= 0.95 a.
// With third derivatives w' (its series converging more slowly) sets the bounds: six terms at
// r >= FAR_D3_K a, five at FAR_D3_K5 a, four at FAR_D3_K4 a (w' within 2e-8, 4e-8, 2e-8).
// FAR_AMAX bounds a so that the FP32 coefficients (~ b a^10) stay finite.
static constexpr double FAR_K = 5.0;
static constexpr double FAR_K5 = 7.0;
static constexpr double FAR_K4 = 13.0;
static constexpr double FAR_D3_K = 6.0;
static constexpr double FAR_D3_K5 = 8.0;
static constexpr double FAR_D3_K4 = 15.0;
static constexpr double FAR_AMAX = 1e3;
// m's term in t^p (p = 2, 3, 5, 7, 9, 11) gives w's in t^(p+2) (factor -p) and w''s in t^(p+4)
// (w' = dw/d(r^2) = -(t^3/2) dw/dt: factor (p + 2) p / 2)
static constexpr float FAR_WP[6] = {4.0f, 7.5f, 17.5f, 31.5f, 49.5f, 71.5f};
struct MemRec64 {
  double x, y, b, s, a, s2, a2, c, sn, q2, e, bqe, bd, apls;
};

// A member table of S samples holds S * n_mem MemRec32 records followed by S blocks, one per
// sample, of the fields the grid tiles classify and expand members with, as structure of arrays
// of soa_pad(n_mem) entries: centre x, y and cut radius a (FP64), then the near-field radius^2
// rn2 and the far-field coefficients fm0..fm5 (FP32).  The 64 lanes of a wave that take 64
// consecutive members read 64 consecutive entries of a field (a few cache lines) instead of one
// field of 64 records 128 bytes apart.
__host__ __device__ inline size_t soa_pad(int n) { return ((size_t)n + 63) / 64 * 64; }
__host__ __device__ inline size_t soa_block_bytes(int n) { return soa_pad(n) * (3 * sizeof(double) + 7 * sizeof(float)); }
__host__ __device__ inline size_t mem32_bytes(int S, int n) {
  return sizeof(MemRec32) * (size_t)S * (size_t)n + (size_t)S * soa_block_bytes(n);
}
struct MemSoA {
  double *x, *y, *a;
  float *rn2, *fm;     // coefficient k of member i: fm[k * pad + i]
  size_t pad;
};
// The block of sample s of a table of S samples of n members.
__host__ __device__ inline MemSoA mem_soa(const MemRec32* m32, int S, int n, int s) {
  MemSoA v;
  v.pad = soa_pad(n);
  char* b = (char*)(m32 + (size_t)S * n) + (size_t)s * soa_block_bytes(n);
  v.x = (double*)b;
  v.y = v.x + v.pad;
  v.a = v.y + v.pad;
  v.rn2 = (float*)(v.a + v.pad);
  v.fm = v.rn2 + v.pad;
  return v;
}

struct SegOff {          // member index range of each segment: [off[k], off[k+1])
  int32_t off[NSEG + 1];
};

}  // namespace lf
