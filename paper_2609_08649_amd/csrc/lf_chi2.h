// Launch interface of the chi^2 kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "lf_device.h"
#include "lf_launch.h"

namespace lf {

struct Chi2Args {
  DevModel m;
  const MainRec* mains;      // [S][n_main]
  const MulRec* muls;        // [S]
  const MemCat32* cat32;     // FP32 member catalog (resident)
  int S, n_img, n_fam;
  const double* th;          // [n_img*2], images sorted by family
  const int* fam;            // [n_img]
  const int* fam_start;      // [n_fam+1]
  const double* afam;        // [n_fam]
  const double* sinv;        // [n_img*3]
  const double* sigmax;      // [n_img]
  double* part;              // [S*n_img*5] alpha, psi at theta_obs
  int* pflags;               // [S*n_img]
  double* wimg;              // [S*n_img*6] W (3), beta_obs (2), det A at theta_obs
  double* csrc;              // [S*n_img] source-plane term of each image
  double* cimg;              // [S*n_img] image-plane term of each image
  int* iflags;               // [S*n_img]
  double* bm_ws;             // [S*n_fam*2] beta_model
  double* chi2;              // [S] out
  int* flags;                // [S] out (may be null)
  double* bmod;              // [S*n_fam*2] out (may be null)
  double* tmod;              // [S*n_img*2] model image positions (may be null)
  double newton_tol;
  // flux and time-delay terms (Sec. 3.2, 3.3); the pointers are null without such data
  const double* mag;         // [n_img] observed magnitudes (sorted order)
  const double* smag;        // [n_img] their errors; <= 0: no measurement
  const double* dt;          // [n_img] observed delays [days]
  const double* sdt;         // [n_img] their errors; <= 0: no measurement
  const double* tsc;         // [n_fam] (1+z_d)/c D_d D_s/D_ds theta_0^2 [days / arcsec^2]
  double* ext;               // [S*n_img*8] FP64 at theta_obs: psi, psi_111..psi_222, psi_11, psi_12, psi_22
  double* extm;              // [S*n_img*4] FP64 at accepted model images: psi, psi_11, psi_12, psi_22
  double* terms;             // [S*3] out: position, flux, delay chi^2 terms (may be null)
  int* strag_n;              // [1] image-plane Newton: number of images left for round 2
  int n_cu;                  // compute units (grid of the round-2 launch)
  Quad qd;
};

// Uneven batches: many (model, constraints, samples) items in one persistent launch.
struct BatchTile {
  int item, pad;
  long long g0, g1;          // thread range [g0, g1) of the item's (image, sample) pairs
};
struct BatchArgs {
  const Chi2Args* items;     // [n_items] (device)
  int n_items;
  const BatchTile* tiles;    // [n_tiles], largest work first
  int n_tiles;
  int* counter;              // [2] tile queues (halo sums, Newton)
  const int* samp_item;      // [total_S] item of each sample of the batch
  const int* samp_local;     // [total_S] its index inside the item
  int total_S;
};

hipError_t launch_batch(const BatchArgs& B, bool mixed, int mode, int block, int grid_persist, hipStream_t st);
hipError_t launch_batch_lean_only(const BatchArgs& B, bool mixed, int block, int grid_persist, hipStream_t st);

hipError_t launch_chi2(const Chi2Args& A, bool mixed, int mode, hipStream_t st,
                       void (*mark)(void*, const char*, int), void* ctx);
// Per-image outputs of an image-plane launch (tmod set): model image positions and image flags
// scattered from the family-sorted order to the caller's constraint order (either may be null).
hipError_t launch_chi2_images_out(const Chi2Args& A, const int* order, double* theta_model, int* img_flags,
                                  hipStream_t st);

}  // namespace lf

