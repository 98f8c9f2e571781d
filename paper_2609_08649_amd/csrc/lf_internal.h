// Internal host/device data layouts of the lensfield library (not part of the ABI).
#pragma once
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

// FP32 copy of the member catalog (centre kept in FP64) for the per-lane scaled chi^2 path.
struct MemCat32 {
  double x, y;
  float fb, fs, fa, q, c, sn, pad0, pad1;
};

// Per-sample member multipliers (b*, s*, a*) and sample validity flags.
struct MulRec {
  double b, s, a;
  int32_t flags, pad;
};

// Pre-scaled member record for one sample.  FP32 flavour keeps the FP64 centre so that
// the offset point - centre is formed exactly before rounding.
struct MemRec32 {
  double x, y;
  float b, s, a, s2, a2, c, sn, q2, e, bqe, pad0, pad1;
};
struct MemRec64 {
  double x, y, b, s, a, s2, a2, c, sn, q2, e, bqe;
};

struct SegOff {          // member index range of each segment: [off[k], off[k+1])
  int32_t off[NSEG + 1];
};

}  // namespace lf
