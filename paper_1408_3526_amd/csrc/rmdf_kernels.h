// rmdf_kernels.h - launch interface between the host library and the gfx950
// kernels of the recursive multidimensional prediction-error filter.
#pragma once
#include <hip/hip_runtime.h>

namespace rmdf {

constexpr int RCX = 256;       // columns per row-kernel block
constexpr int RSEG = 16;       // columns per resonator segment (direct-DFT seed at its start)
constexpr int NVY_MAX = 33;    // largest candidate grid per axis
constexpr int NVX_MAX = 33;

// Arguments of the per-pixel kernel (passed by value).
struct PixArgs {
  int H, W, TY;                // frame size, rows per work tile
  int nvx, nvy, nv;            // candidate grid
  int bx, by, dx, dy;          // half-bandwidth, spatial output delay
  int vmode;                   // 0 search, 2 fixed velocity, 3 search refined between grid points
  float alpha, inv_sqrt_my;
  float fvx, fvy;
  const float2* rs;            // row spectra [H][W][planes]
  float2* st;                  // observer state [H][W][planes*My][Mz] (16x16x8 wave-per-anchor
                               // kernel: [H][W][Mz/2][planes*My][2])
  float* rsm;                  // smoothed autocorrelation [H][W][nv]
  const float* ring_delayed;   // input frame t - m'_t, or nullptr while t < m'_t
  float* out;                  // [H][W]
  float2* vxy;                 // [H][W]
  int* vidx;                   // [H][W]
  const float2* twy;           // [My]  w_y^k
  const float2* twz;           // [Mz]  w_z^k
  const float2* twA;           // [Mz]  stage-A weights (w_z^k and scale)
  const float2* tauy;          // [nvy][My]  trigonometric weights along ky
  const float2* taux;          // [nvx][Mx/2+1] weights along kx (Hermitian factor folded)
  const float2* htab;          // [nv+1][bx+1][2by+1][Mz] background coefficients
  const float* gx;             // [nvx]
  const float* gy;             // [nvy]
  const float* tabB;           // [nvy][16] cos/sin(2 pi k l_y / 16), k = 1..7; cos(pi l_y)
  const float* tabC;           // [nvx][16] 2cos/2sin(2 pi k l_x / 16), k = 1..7; cos(pi l_x)
  unsigned short* feat;        // [H][W][9][16][8] BF16 learned-model features (16x16x8), or nullptr
  int* fidx;                   // [H][W] search index for the learned-mode fallback
  int dt;                      // temporal output delay
  // Lattice form of the background coefficients (16x16x8 kernel): when every
  // candidate velocity v satisfies v*s integral for s in {1, 2, 4}, the
  // coefficient at (kx, ky, kz) factors as etab[kx][ky+by] * gtab[q][kz] with
  // q = (nx kx + ny ky) mod 16s, (nx, ny) = s*v.  gtab == nullptr: no lattice.
  const float2* gtab;          // [16s][Mz]
  const float2* etab;          // [bx+1][2by+1]
  const int* latq;             // [nv+1] (nx << 16) | (ny & 0xffff); entry nv = fixed velocity
  int lat_q;                   // 16s
  int tcur;                    // index of the frame being pushed (ring slot = tcur mod Mz)
  // frame pairs (16x16x8 kernel, mode 6): the second frame's row spectra and
  // delayed input; the first frame's output goes to out_first
  const float2* rs2;
  const float* ring_delayed2;
  float* out_first;
};

bool shape_supported(int mx, int my, int mz);
int planes_for(int mx);
// anchors (columns) one workgroup of the generic pixel kernel covers per row
int pixel_block_columns(int mx, int my, int mz);
// default rows per work tile for an H x W frame
int auto_tile_rows(int H, int W, int block_columns);
hipError_t launch_pixel(int mx, int my, int mz, const PixArgs& a, hipStream_t s);
// row sliding DFT of the frame f; also copies f into the delay-ring slot
// (non-finite samples zeroed and counted in *nonfinite).  direct: each output
// is the direct DFT sum of its window instead (Mx = 16 only)
hipError_t launch_row(int mx, const float* f, float2* rs, const float2* twx, int H, int W, float* slot,
                      unsigned long long* nonfinite, hipStream_t s, bool direct = false);
// layout: 0 generic observer state [plane][ky][kz]; 1 wave-per-anchor 16x16x8
// observer state; 2 ring of 2-D spectra [slot][plane][ky] whose newest frame
// is `newest` (slot newest mod Mz)
hipError_t launch_spectrum(int mx, int my, int mz, const float2* st, int W, const int* xy, int npix, float2* out,
                           int layout, int newest, hipStream_t s);
bool pixel16_eligible(int mx, int my, int mz, int nvx, int nvy);
int p16_block_columns();   // anchors per workgroup of the 16x16x8 wave-per-anchor kernel
// mode: 0 search (or fixed velocity), 1 search + learned features, 2 learned
// first pass, 3 search refined between grid points, 4 search (or fixed
// velocity) with the ring of 2-D spectra in place of the observer state, 5 as
// 4 with the column DFT summed directly (no recursion on any axis), 6 as 0 for
// two frames in one pass over the state (rs: first frame, rs2: second)
hipError_t launch_pixel16(const PixArgs& a, int mode, hipStream_t s);
// learned mode: zero the confident-anchor count list[0] (before the network
// kernel appends to the list), then filter the listed anchors
hipError_t launch_conf_reset(int* list, hipStream_t s);
hipError_t launch_finish16(const PixArgs& a, const float* vc, float thr, const int* list, hipStream_t s);

}  // namespace rmdf
