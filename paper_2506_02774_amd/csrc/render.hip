// Splatting kernels (gfx950): Section 3.1 "Culling & Projection", "Sorting"
// and "Rasterization", with the preemptive alpha-filtering of Section 4.2.
//
//   render_setup  zero the frame's counters, digit histograms and tile ranges
//   project       EWA projection + SH colour per cut Gaussian, tile rect,
//                 pair count (alpha filter: Eq. 4 per Gaussian / rect / tile),
//                 depth key + its 4 digit histograms
//   depth sort    4 stable onesweep passes over 8-bit digits of the depth bits
//                 (values = cut positions, so equal depths keep node-id order)
//   emit          exclusive scan of the pair counts in depth order fused with
//                 the emission of the Gaussian-tile pairs (tile key + cut
//                 position) + the tile digit histograms; big Gaussians by
//                 whole workgroups
//   tile sort     2 stable onesweep passes on the tile id: afterwards pairs are
//                 ordered by (tile, depth, node id) - an LSD radix sort by
//                 (tile, depth) whose depth digits were sorted before the
//                 Gaussians were replicated into pairs
//   ranges        [start, end) of every tile in the sorted pairs
//   blend         one 256-thread workgroup per 16x16 tile, Gaussians staged in
//                 LDS in batches of 256, front-to-back alpha blending (Eq. 3)
#include <mutex>
#include <new>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "sort.hpp"
#include "vy_common.hpp"

#pragma clang fp contract(off)


namespace {

using namespace vyd;

constexpr int kTileSize = 16;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kLowpass = 0.3f;
constexpr float kClamp = 1.3f;
constexpr float kRadiusK = 3.33f;        // > sqrt(2 ln 255) = 3.32904: alpha < 1/255 beyond it
constexpr uint32_t kBigArea = 32;        // rects with more tiles are binned by a whole workgroup
constexpr float kFilterDelta = 1e-3f;    // margin of the preemptive check (keeps it lossless)

// ctr layout
enum {
  C_NVIS = 0,      // Gaussians that produce at least one pair
  C_NPAIRS = 1,    // pairs stored (clamped to capacity)
  C_NPAIRS_RAW = 2,
  C_ERR = 3,
  C_TICKET0 = 4,   // 4..9 sort passes, 10 scan
  C_SCAN_TICKET = 10,
  C_OVERFLOW = 11,
  C_NBIG = 12,     // Gaussians whose rect exceeds kBigArea tiles
  C_NHEAVY = 13,   // tiles split over several jobs
  C_NJOBS = 14,    // blend jobs of split tiles
  C_SLOTS = 15,    // per-bin result slots handed out
  C_JOB_TICKET = 16,
  C_NREDO = 17,    // (heavy tile, bin) units with pixels that stop in the bin
  C_NTIER = 18,    // 18..20: tiles in the heavy-first tiers
  C_BAND_TICKET = 21,   // wave-level band jobs of the two heaviest tiers
  C_GOVER = 22,    // cut size when it exceeds the context's max_gaussians (else 0)
  C_COUNT = 32
};

struct RCam {
  float R[9];
  float px, py, pz;
  float fx, fy, cx, cy;
  float near;
  float ulo, uhi, vlo, vhi;  // clamp range of x/z and y/z
  int W, H, tiles_x, tiles_y;
  float bg[3];
  float ln_amin;             // log(1/255)
  float fdelta;              // margin of the preemptive check (wider with the LUT)
};

// One viewer's frame in a batch rendered with one launch per stage: its
// camera, scene records, cut, image, and where its Gaussians and tiles start
// in the batch (cut positions [g_off[v], g_off[v + 1]) of the concatenated
// cuts, global tiles [tile_base, tile_base + tiles_x * tiles_y)).
struct BView {
  RCam cam;
  const float4* gauss;
  const float* sh;
  const int32_t* cut;
  const int32_t* n_cut;   // device count of the view's cut
  int64_t n_nodes;
  float* img;
  uint32_t tile_base;
  uint32_t pad;
};
constexpr int kMaxViews = 64;

// The view holding batch position i: the largest v with off[v] <= i (off has
// nv + 1 ascending entries, off[0] = 0).
VY_DEV int view_of(const uint32_t* off, int nv, uint32_t i) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Per-Gaussian view data of a batched launch (BATCH), or the single frame's.
struct ViewsRef {
  const BView* views;      // device
  const uint32_t* g_off;   // device [nv + 1]: first batch position of each view
  int nv;
};

__global__ void render_setup(uint32_t* ctr, uint32_t* hist, uint2* ranges, int ntiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int i = t; i < C_COUNT; i += stride) ctr[i] = 0;
  for (int i = t; i < 6 * 256; i += stride) hist[i] = 0;
  for (int i = t; i < ntiles; i += stride) ranges[i] = make_uint2(0, 0);
}

// Real SH, degree <= 3, orthonormal, no Condon-Shortley phase; index l*l+l+m.
VY_DEV float3 sh_colour(const float* __restrict__ c, float x, float y, float z) {
  const float C0 = 0.28209479177387814f;
  const float C1 = 0.4886025119029199f;
  const float C2a = 1.0925484305920792f;   // xy, yz, xz
  const float C20 = 0.31539156525252005f;  // 3z^2 - 1
  const float C22 = 0.5462742152960396f;   // x^2 - y^2
  const float C33 = 0.5900435899266435f;   // y(3x^2 - y^2), x(x^2 - 3y^2)
  const float C32 = 2.890611442640554f;    // xyz
  const float C31 = 0.4570457994644658f;   // y(5z^2 - 1), x(5z^2 - 1)
  const float C30 = 0.3731763325901154f;   // z(5z^2 - 3)
  const float C32p = 1.445305721320277f;   // z(x^2 - y^2)
  const float xx = x * x, yy = y * y, zz = z * z;
  float Y[16];
  Y[0] = C0;
  Y[1] = C1 * y;
  Y[2] = C1 * z;
  Y[3] = C1 * x;
  Y[4] = C2a * (x * y);
  Y[5] = C2a * (y * z);
  Y[6] = C20 * (3.f * zz - 1.f);
  Y[7] = C2a * (x * z);
  Y[8] = C22 * (xx - yy);
  Y[9] = C33 * y * (3.f * xx - yy);
  Y[10] = C32 * (x * y) * z;
  Y[11] = C31 * y * (5.f * zz - 1.f);
  Y[12] = C30 * z * (5.f * zz - 3.f);
  Y[13] = C31 * x * (5.f * zz - 1.f);
  Y[14] = C32p * z * (xx - yy);
  Y[15] = C33 * x * (xx - 3.f * yy);
  float r = 0.f, g = 0.f, b = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    r = fmaf(Y[k], c[3 * k + 0], r);
    g = fmaf(Y[k], c[3 * k + 1], g);
    b = fmaf(Y[k], c[3 * k + 2], b);
  }
  return make_float3(fminf(fmaxf(r + 0.5f, 0.f), 1.f), fminf(fmaxf(g + 0.5f, 0.f), 1.f),
                     fminf(fmaxf(b + 0.5f, 0.f), 1.f));
}

// Maximum of rho(d) = A d_x^2 + B d_x d_y + C d_y^2 (A, C < 0: the power of a
// Gaussian, d = pixel centre - mean) over pixel centres spanning [x0, x1] x
// [y0, y1] (a tile, or the band of a band job): the exact maximum over the
// continuous rectangle (0 if the mean is inside, else the best of the four
// edges, each a 1-D concave quadratic maximised at its clamped vertex).
VY_DEV float rect_rho_max(float mx, float my, float A, float B, float C, float x0, float y0, float x1, float y1) {
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.f;
  const float dx0 = x0 - mx, dx1 = x1 - mx, dy0 = y0 - my, dy1 = y1 - my;
  float best = -INFINITY;
  for (int e = 0; e < 2; ++e) {  // edges with d_x fixed
    const float dx = e ? dx1 : dx0;
    const float dy = fminf(fmaxf(-B * dx / (2.f * C), dy0), dy1);
    best = fmaxf(best, (A * dx * dx + C * dy * dy) + B * dx * dy);
  }
  for (int e = 0; e < 2; ++e) {  // edges with d_y fixed
    const float dy = e ? dy1 : dy0;
    const float dx = fminf(fmaxf(-B * dy / (2.f * A), dx0), dx1);
    best = fmaxf(best, (A * dx * dx + C * dy * dy) + B * dx * dy);
  }
  return fminf(best, 0.f);
}

VY_DEV float tile_rho_max(float mx, float my, float A, float B, float C, int tx, int ty, int W, int H) {
  const float x0 = tx * kTileSize + 0.5f, y0 = ty * kTileSize + 0.5f;
  const float x1 = fminf((float)(tx * kTileSize + kTileSize), (float)W) - 0.5f;
  const float y1 = fminf((float)(ty * kTileSize + kTileSize), (float)H) - 0.5f;
  return rect_rho_max(mx, my, A, B, C, x0, y0, x1, y1);
}

// Pair-level preemptive test (Eq. 4 moved to binning, Section 4.2): keep tile t
// unless every pixel centre in it has rho below thr. `relax` >= 0 is a relative
// allowance for float32 rounding of the per-pixel rho (grows with the conic's
// condition number) so that a dropped pair could never have been blended.
VY_DEV bool tile_keep(const float4 p0, const float4 p1, float relax, int tx, int ty, int W, int H) {
  const float rm = tile_rho_max(p0.x, p0.y, p0.z, p0.w, p1.x, tx, ty, W, H);
  return rm * (1.f - relax) >= p1.z;
}

// The pixel box of a Gaussian (centre (mx, my), half-extents rx, ry) within
// the first and last tile columns and rows of its tile rect [x0, x1] x [y0, y1]:
// the first column of tile x0 and the last of tile x1 (and likewise for
// rows) that may hold a pixel centre passing the pixel rule, clamped to the
// tile. Column px passes when |mx - (px + 0.5)| <= rx, so the columns are
// ceil(mx - rx - 0.5) .. floor(mx + rx - 0.5). The slack, 1/8 px plus
// 2^-19 (|mx| + rx), is over 4x the rounding of these sums and of the rule's
// own difference (about 2^-22 (|mx| + rx + 2^15) in all), so the box is a
// superset at any centre and extent. 4 bits each:
// first column | last column << 4 | first row << 8 | last row << 12. Tiles
// between the first and last take every column (row); a pair's key carries
// its own tile's range (pair_emit), so that band jobs can tell which pairs
// may reach their band from the sorted keys alone.
VY_DEV uint32_t pixel_box(float mx, float my, float rx, float ry, int x0, int y0, int x1, int y1) {
  const float sx = 0.125f + (fabsf(mx) + rx) * 0x1p-19f, sy = 0.125f + (fabsf(my) + ry) * 0x1p-19f;
  const int px0 = (int)ceilf(mx - rx - 0.5f - sx), px1 = (int)floorf(mx + rx - 0.5f + sx);
  const int py0 = (int)ceilf(my - ry - 0.5f - sy), py1 = (int)floorf(my + ry - 0.5f + sy);
  const uint32_t a = (uint32_t)min(max(px0 - x0 * kTileSize, 0), kTileSize - 1);
  const uint32_t b = (uint32_t)min(max(px1 - x1 * kTileSize, 0), kTileSize - 1);
  const uint32_t c = (uint32_t)min(max(py0 - y0 * kTileSize, 0), kTileSize - 1);
  const uint32_t d = (uint32_t)min(max(py1 - y1 * kTileSize, 0), kTileSize - 1);
  return a | (b << 4) | (c << 8) | (d << 12);
}
constexpr uint32_t kWholeTileBox = 0xF0F0u;   // columns 0..15, rows 0..15

// The pair count of a binning record's (mask, count word): rects of at most
// kBigArea tiles (mask != 0) keep the count in the low 8 bits and the pixel
// box above it; big rects keep the whole word for their count.
VY_DEV uint32_t rec_count(uint2 mask_count) { return mask_count.x ? (mask_count.y & 0xFFu) : mask_count.y; }

// The pixel box of a pair's tile (tx, ty) as key bits 16..31 (pair_emit).
VY_DEV uint32_t pair_box_bits(uint32_t box, int tx, int ty, int x0, int y0, int x1, int y1) {
  const uint32_t lx = tx == x0 ? (box & 15u) : 0u, hx = tx == x1 ? ((box >> 4) & 15u) : 15u;
  const uint32_t ly = ty == y0 ? ((box >> 8) & 15u) : 0u, hy = ty == y1 ? ((box >> 12) & 15u) : 15u;
  return (lx | (hx << 4) | (ly << 8) | (hy << 12)) << 16;
}

// One cut Gaussian (cut position i, node id `node`): EWA projection, SH
// colour, pixel extents, tile rect and (FILTER) the Eq. 4 tests; writes its
// records at position i and returns its depth key (0xFFFFFFFF when culled) and
// pair count. Rects of more than kBigArea tiles are appended to `big`.
template <bool FILTER>
VY_DEV uint32_t project_one(uint32_t i, int32_t node, const float4* __restrict__ gauss, const float* __restrict__ sh,
                            const RCam& cam, float4* __restrict__ pg0, float4* __restrict__ pg1,
                            float4* __restrict__ pg2, uint4* __restrict__ prec, float* __restrict__ prelax,
                            uint32_t* ctr, uint32_t* __restrict__ big, uint32_t* count_out) {
  const float4 g0 = gauss[3 * (int64_t)node], g1 = gauss[3 * (int64_t)node + 1], g2 = gauss[3 * (int64_t)node + 2];
  const float dxw = g0.x - cam.px, dyw = g0.y - cam.py, dzw = g0.z - cam.pz;
  const float x = (cam.R[0] * dxw + cam.R[1] * dyw) + cam.R[2] * dzw;
  const float y = (cam.R[3] * dxw + cam.R[4] * dyw) + cam.R[5] * dzw;
  const float z = (cam.R[6] * dxw + cam.R[7] * dyw) + cam.R[8] * dzw;
  bool valid = z > cam.near;
  uint32_t count = 0, mask = 0, key = 0xFFFFFFFFu;
  float4 o0 = make_float4(0, 0, 0, 0), o1 = make_float4(0, 0, 0, 0), o2 = make_float4(0, 0, 0, 0);
  uint32_t r0 = 0, r1 = 0, box = 0;
  float relax = 0.f;
  if (valid) {
    // Sigma3 = M M^T with M = Rq diag(s)
    const float qw = g2.x, qx = g2.y, qy = g2.z, qz = g2.w;
    const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                         2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                         2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    const float s[3] = {g1.x, g1.y, g1.z};
    const float iz = 1.f / z;
    const float u = fminf(fmaxf(x * iz, cam.ulo), cam.uhi);
    const float v = fminf(fmaxf(y * iz, cam.vlo), cam.vhi);
    // T = J R (2x3): rows fx/z (R0 - u R2), fy/z (R1 - v R2)
    float T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
      T0[k] = (cam.fx * iz) * (cam.R[k] - u * cam.R[6 + k]);
      T1[k] = (cam.fy * iz) * (cam.R[3 + k] - v * cam.R[6 + k]);
    }
    // V = T M (2x3); Sigma2 = V V^T + lowpass
    float V0[3], V1[3];
    for (int j = 0; j < 3; ++j) {
      const float m0 = Rq[0 + j] * s[j], m1 = Rq[3 + j] * s[j], m2 = Rq[6 + j] * s[j];
      V0[j] = (T0[0] * m0 + T0[1] * m1) + T0[2] * m2;
      V1[j] = (T1[0] * m0 + T1[1] * m1) + T1[2] * m2;
    }
    const float a = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + kLowpass;
    const float b = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2];
    const float c = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + kLowpass;
    const float det = fmaf(a, c, -b * b);
    valid = det > 0.f;
    if (valid) {
      const float idet = 1.f / det;
      const float ca = c * idet, cb = -b * idet, cc = a * idet;
      const float mx = cam.fx * x * iz + cam.cx, my = cam.fy * y * iz + cam.cy;
      const float mid = 0.5f * (a + c);
      const float lmax = mid + sqrtf(fmaxf(0.f, mid * mid - det));
      const float lmin = fmaxf(det / lmax, 1e-30f);
      // per-axis extents: the ellipse d^T Sigma2^-1 d <= K^2 (outside it alpha < 1/255)
      // lies within |dx| <= K sqrt(Sigma2_xx), |dy| <= K sqrt(Sigma2_yy)
      float rx = fminf(ceilf(kRadiusK * sqrtf(a)), 65535.f), ry = fminf(ceilf(kRadiusK * sqrtf(c)), 65535.f);
      const float theta = g1.w, log_theta = g0.w;
      const float thr = cam.ln_amin - log_theta - cam.fdelta;
      // relative rounding bound of rho for this conic (condition number based)
      relax = 1e-6f * (lmax / lmin);
      if (FILTER) {
        if (thr > 0.f) valid = false;      // theta below alpha*: never blended
        if (valid && relax < 0.25f) {
          // outside the box of the ellipse rho >= thr every pixel has rho < thr
          // (margins for the rounding of the conic and of the per-pixel rho)
          const float f = 2.f * (-thr) * ((1.f + relax) / (1.f - relax)) * 1.001f;
          rx = fminf(rx, ceilf(sqrtf(f * a + 2.f)));
          ry = fminf(ry, ceilf(sqrtf(f * c + 2.f)));
        }
      }
      if (valid) {
        int x0 = (int)floorf((mx - rx) / kTileSize), x1 = (int)floorf((mx + rx) / kTileSize);
        int y0 = (int)floorf((my - ry) / kTileSize), y1 = (int)floorf((my + ry) / kTileSize);
        x0 = max(x0, 0);
        y0 = max(y0, 0);
        x1 = min(x1, cam.tiles_x - 1);
        y1 = min(y1, cam.tiles_y - 1);
        if (x0 > x1 || y0 > y1) valid = false;
        if (valid) {
          // rho = A dx^2 + B dx dy + C dy^2 with (A, B, C) = (-a/2, -b, -c/2) of the conic
          o0 = make_float4(mx, my, -0.5f * ca, -cb);
          o1 = make_float4(-0.5f * cc, theta, thr, z);
          const float dn = 1.f / sqrtf((dxw * dxw + dyw * dyw) + dzw * dzw);
          const float3 rgb = sh_colour(sh + 48 * (int64_t)node, dxw * dn, dyw * dn, dzw * dn);
          o2 = make_float4(rgb.x, rgb.y, rgb.z, __uint_as_float((uint32_t)rx | ((uint32_t)ry << 16)));
          r0 = (uint32_t)x0 | ((uint32_t)y0 << 16);
          r1 = (uint32_t)x1 | ((uint32_t)y1 << 16);
          const uint32_t area = (uint32_t)(x1 - x0 + 1) * (uint32_t)(y1 - y0 + 1);
          if (area > kBigArea) {
            // binned by a whole workgroup (big_count / emit_big); with the filter
            // the count is provisional until big_count applies the tile test
            count = area;
            big[fetch_add(ctr + C_NBIG, 1u)] = i;
          } else if (FILTER && relax < 0.25f) {
            uint32_t bit = 1u;
            for (int ty = y0; ty <= y1; ++ty)
              for (int tx = x0; tx <= x1; ++tx, bit <<= 1)
                if (tile_keep(o0, o1, relax, tx, ty, cam.W, cam.H)) mask |= bit;
            count = (uint32_t)__popc(mask);
          } else {
            count = area;
            mask = area == 32u ? 0xFFFFFFFFu : (1u << area) - 1u;
          }
          if (count == 0) valid = false;
          else key = __float_as_uint(z);
          if (valid && area <= kBigArea) box = pixel_box(mx, my, rx, ry, x0, y0, x1, y1);
        }
      }
    }
  }
  if (!valid) count = mask = box = 0;
  pg0[i] = o0;
  pg1[i] = o1;
  pg2[i] = o2;
  prec[i] = make_uint4(r0, r1, mask, count | (box << 8));
  prelax[i] = relax;
  *count_out = count;
  return key;
}

// Histograms of the 4 depth digits and the count of visible Gaussians, per
// block, flushed with one atomic per non-zero bin.
VY_DEV void project_flush(uint32_t (*s_hist)[256], uint32_t nvis, uint32_t* ctr, uint32_t* hist) {
  for (int o = 32; o > 0; o >>= 1) nvis += __shfl_xor(nvis, o, 64);
  if (lane() == 0 && nvis) atomicAdd(ctr + C_NVIS, nvis);
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
    const uint32_t v = (&s_hist[0][0])[i];
    if (v) atomicAdd(hist + i, v);
  }
}

template <bool FILTER>
__global__ __launch_bounds__(256) void project(const int32_t* __restrict__ cut, const int32_t* n_cut_ptr,
                                               const float4* __restrict__ gauss, const float* __restrict__ sh,
                                               RCam cam, float4* __restrict__ pg0, float4* __restrict__ pg1,
                                               float4* __restrict__ pg2, uint4* __restrict__ prec,
                                               float* __restrict__ prelax, uint32_t* __restrict__ dkey,
                                               uint32_t* ctr, uint32_t* hist, int64_t n_nodes,
                                               uint32_t* __restrict__ big, uint32_t gcap) {
  __shared__ uint32_t s_hist[4][256];
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&s_hist[0][0])[i] = 0;
  __syncthreads();
  const uint32_t n_all = (uint32_t)*n_cut_ptr;
  // a cut larger than the context renders its first gcap entries and is reported
  if (n_all > gcap && blockIdx.x == 0 && threadIdx.x == 0) ctr[C_GOVER] = n_all;
  const int64_t n = n_all < gcap ? n_all : gcap;
  uint32_t nvis = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t node = cut[i];
    if (node < 0 || node >= n_nodes) node = 0;
    uint32_t count;
    const uint32_t key = project_one<FILTER>((uint32_t)i, node, gauss, sh, cam, pg0, pg1, pg2, prec, prelax, ctr, big,
                                             &count);
    dkey[i] = key;
    nvis += count > 0 ? 1u : 0u;
#pragma unroll
    for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
  }
  project_flush(s_hist, nvis, ctr, hist);
}

// Batched frames: counters, histograms and tile ranges cleared, and the
// views' first batch positions (prefix sums of their cut sizes, the total
// clamped to the context's capacity, an overflow recorded in C_GOVER).
__global__ void batch_setup(const BView* __restrict__ views, int nv, uint32_t* __restrict__ g_off, uint32_t gcap,
                            uint32_t* ctr, uint32_t* hist, uint2* ranges, int ntiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int i = t; i < C_COUNT; i += stride)
    if (i != C_GOVER) ctr[i] = 0;
  for (int i = t; i < 6 * 256; i += stride) hist[i] = 0;
  for (int i = t; i < ntiles; i += stride) ranges[i] = make_uint2(0, 0);
  if (t == 0) {
    uint64_t acc = 0;
    for (int v = 0; v < nv; ++v) {
      g_off[v] = (uint32_t)(acc < gcap ? acc : gcap);
      const int32_t c = *views[v].n_cut;
      acc += c > 0 ? (uint64_t)c : 0ull;
    }
    g_off[nv] = (uint32_t)(acc < gcap ? acc : gcap);
    ctr[C_GOVER] = acc > gcap ? (uint32_t)(acc < 0xFFFFFFFFull ? acc : 0xFFFFFFFFull) : 0u;
  }
}

// Projection of the concatenated cuts of a batch of views (each Gaussian with
// its own view's scene, camera and filter), into batch positions.
template <bool FILTER>
__global__ __launch_bounds__(256) void project_batch(const BView* __restrict__ views, const uint32_t* __restrict__ g_off,
                                                     int nv, float4* __restrict__ pg0, float4* __restrict__ pg1,
                                                     float4* __restrict__ pg2, uint4* __restrict__ prec,
                                                     float* __restrict__ prelax, uint32_t* __restrict__ dkey,
                                                     uint32_t* ctr, uint32_t* hist, uint32_t* __restrict__ big) {
  __shared__ uint32_t s_hist[4][256];
  __shared__ uint32_t s_off[kMaxViews + 1];
  __shared__ RCam s_cam[kMaxViews];
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&s_hist[0][0])[i] = 0;
  for (int v = threadIdx.x; v <= nv; v += blockDim.x) s_off[v] = g_off[v];
  for (int v = threadIdx.x; v < nv; v += blockDim.x) s_cam[v] = views[v].cam;
  __syncthreads();
  const uint32_t n = s_off[nv];
  uint32_t nvis = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = view_of(s_off, nv, i);
    const BView& V = views[v];
    int32_t node = V.cut[i - s_off[v]];
    if (node < 0 || node >= V.n_nodes) node = 0;
    uint32_t count;
    const uint32_t key = project_one<FILTER>(i, node, V.gauss, V.sh, s_cam[v], pg0, pg1, pg2, prec, prelax, ctr, big,
                                             &count);
    dkey[i] = key;
    nvis += count > 0 ? 1u : 0u;
#pragma unroll
    for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
  }
  project_flush(s_hist, nvis, ctr, hist);
}

// Filtered pair count of the big Gaussians: one workgroup per Gaussian, its
// rect's tiles spread over the threads.
template <bool BATCH>
__global__ __launch_bounds__(256) void big_count(const uint32_t* __restrict__ big, const uint32_t* ctr,
                                                 const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                                                 uint4* __restrict__ prec, const float* __restrict__ prelax,
                                                 int W, int H, uint32_t n_g, ViewsRef vr) {
  __shared__ uint32_t s_red[4];
  const uint32_t nb = ctr[C_NBIG];
  for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint32_t g = big[b];
    if (g >= n_g) continue;
    if (BATCH) {
      const int v = view_of(vr.g_off, vr.nv, g);
      W = vr.views[v].cam.W;
      H = vr.views[v].cam.H;
    }
    const uint4 r = prec[g];
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
    const int w = x1 - x0 + 1, area = w * (y1 - y0 + 1);
    const float4 p0 = pg0[g], p1 = pg1[g];
    const float relax = prelax[g];
    uint32_t cnt = 0;
    for (int k = threadIdx.x; k < area; k += blockDim.x)
      cnt += (relax >= 0.25f || tile_keep(p0, p1, relax, x0 + k % w, y0 + k / w, W, H)) ? 1u : 0u;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane() == 0) s_red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) reinterpret_cast<uint32_t*>(prec + g)[3] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    __syncthreads();
  }
}

// Pair scan and emission (Section 3.1 "Sorting": one (tile, Gaussian) pair
// per tile a Gaussian touches; with the filter, per the Eq. 4 tile test taken
// in project). The visible Gaussians, in depth order (r < n_vis), get
// consecutive ranges of the pair array by an exclusive scan of their pair
// counts (decoupled look-back over partitions of kScanTile), and each writes
// its pairs in row-major tile order from its kept-tile mask, so the array
// comes out in (depth, node id) order for the stable tile sort. Big Gaussians
// only get their offset here (offs[g]); emit_big writes their pairs. The total
// goes to C_NPAIRS_RAW, min(total, cap) to C_NPAIRS.
constexpr int kScanItems = 12, kScanTile = 256 * kScanItems;   // 8, 16, 24, 32 measured slower

template <bool BATCH>
__global__ __launch_bounds__(256) void pair_emit(const uint32_t* __restrict__ sorted_val,
                                                 const uint4* __restrict__ prec, uint32_t* __restrict__ offsets,
                                                 uint32_t* ctr, uint64_t* status, uint32_t epoch, int tiles_x,
                                                 int bits0, uint32_t* __restrict__ tkey, uint32_t* __restrict__ tval,
                                                 uint32_t* hist, uint32_t cap, uint32_t n_g, ViewsRef vr) {
  __shared__ uint32_t s_v[kScanTile];
  __shared__ uint32_t s_scan[8], s_part;
  __shared__ uint64_t s_ex;
  __shared__ uint32_t s_hist[2][256];
  __shared__ uint32_t s_off[BATCH ? kMaxViews + 1 : 1], s_tx[BATCH ? kMaxViews : 1], s_tb[BATCH ? kMaxViews : 1];
  for (int i = threadIdx.x; i < 512; i += blockDim.x) (&s_hist[0][0])[i] = 0;
  if (BATCH) {
    for (int v = threadIdx.x; v <= vr.nv; v += blockDim.x) s_off[v] = vr.g_off[v];
    for (int v = threadIdx.x; v < vr.nv; v += blockDim.x) {
      s_tx[v] = (uint32_t)vr.views[v].cam.tiles_x;
      s_tb[v] = vr.views[v].tile_base;
    }
  }
  const uint32_t n = ctr[C_NVIS];
  const uint32_t n_parts = (n + kScanTile - 1) / kScanTile;
  const uint32_t m0 = (1u << bits0) - 1u;
  for (;;) {
    if (threadIdx.x == 0) s_part = fetch_add(ctr + C_SCAN_TICKET, 1u);
    __syncthreads();
    const uint32_t part = s_part;
    if (part >= n_parts) break;
    const uint32_t base = part * kScanTile;
    for (int k = 0; k < kScanItems; ++k) {
      const uint32_t i = base + k * 256 + threadIdx.x;
      uint32_t v = 0;
      if (i < n) {
        const uint32_t g = sorted_val[i];
        if (g < n_g) v = rec_count(reinterpret_cast<const uint2*>(prec + g)[1]);
      }
      s_v[k * 256 + threadIdx.x] = v;
    }
    __syncthreads();
    uint32_t loc[kScanItems], sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
      loc[k] = sum;
      sum += s_v[threadIdx.x * kScanItems + k];
    }
    uint32_t tot;
    const uint32_t off = block_excl_scan256(sum, s_scan, &tot);
    if (threadIdx.x < 64) {
      const uint64_t e = lookback_wave(status, part, 1, epoch, tot, ctr + C_ERR);
      if (threadIdx.x == 0) s_ex = e;
    }
    __syncthreads();
    const uint64_t ex = s_ex;
    for (int k = 0; k < kScanItems; ++k) s_v[threadIdx.x * kScanItems + k] = (uint32_t)(ex + off + loc[k]);
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
      const uint32_t i = base + k * 256 + threadIdx.x;
      if (i >= n) continue;
      const uint32_t g = sorted_val[i];
      if (g >= n_g) continue;
      const uint4 r = prec[g];
      if (rec_count(make_uint2(r.z, r.w)) == 0) continue;
      uint32_t o = s_v[k * 256 + threadIdx.x];
      if (r.z == 0) {   // big: emit_big writes its pairs
        offsets[g] = o;
        continue;
      }
      const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16, w = x1 - x0 + 1;
      const uint32_t box = r.w >> 8;
      const uint64_t wmask = (1ull << w) - 1ull;
      uint64_t bits = r.z;
      int tx_n = tiles_x;
      uint32_t tbase = 0;
      if (BATCH) {
        const int v = view_of(s_off, vr.nv, g);
        tx_n = (int)s_tx[v];
        tbase = s_tb[v];
      }
      for (int ty = y0; bits; ++ty, bits >>= w) {
        uint32_t rb = (uint32_t)(bits & wmask);
        while (rb) {
          const int b = __ffs(rb) - 1;
          rb &= rb - 1;
          const uint32_t t = tbase + (uint32_t)(ty * tx_n + x0 + b);
          if (o < cap) {
            tkey[o] = t | pair_box_bits(box, x0 + b, ty, x0, y0, x1, y1);
            tval[o] = g;
            atomicAdd(&s_hist[0][t & m0], 1u);
            atomicAdd(&s_hist[1][(t >> bits0) & 255u], 1u);
          }
          ++o;
        }
      }
    }
    if (part == n_parts - 1 && threadIdx.x == 0) {
      const uint64_t total = ex + tot;
      ctr[C_NPAIRS_RAW] = (uint32_t)(total > 0xFFFFFFFFull ? 0xFFFFFFFFull : total);
      ctr[C_NPAIRS] = (uint32_t)(total > cap ? cap : total);
      if (total > cap) ctr[C_OVERFLOW] = 1;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 512; i += blockDim.x) {
    const uint32_t v = (&s_hist[0][0])[i];
    if (v) atomicAdd(hist + 4 * 256 + i, v);
  }
}

// Pair emission of the big Gaussians: one workgroup per Gaussian; the kept
// tiles of each 256-tile chunk are placed by a block scan (row-major order).
template <bool FILTER, bool BATCH>
__global__ __launch_bounds__(256) void emit_big(const uint32_t* __restrict__ big, const uint32_t* __restrict__ offs,
                                                const uint4* __restrict__ prec,
                                                const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                                                const float* __restrict__ prelax, int W, int H, int tiles_x,
                                                int bits0, uint32_t* __restrict__ tkey, uint32_t* __restrict__ tval,
                                                uint32_t* ctr, uint32_t* hist, uint32_t cap, uint32_t n_g,
                                                ViewsRef vr) {
  __shared__ uint32_t s_hist[2][256];
  __shared__ uint32_t s_scan[8];
  for (int i = threadIdx.x; i < 512; i += blockDim.x) (&s_hist[0][0])[i] = 0;
  __syncthreads();
  const uint32_t nb = ctr[C_NBIG];
  const uint32_t m0 = (1u << bits0) - 1u;
  for (uint32_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const uint32_t g = big[bi];
    if (g >= n_g) continue;
    const uint4 r = prec[g];
    if (r.w == 0) continue;   // uniform over the block
    uint32_t tbase = 0;
    if (BATCH) {
      const int v = view_of(vr.g_off, vr.nv, g);
      W = vr.views[v].cam.W;
      H = vr.views[v].cam.H;
      tiles_x = vr.views[v].cam.tiles_x;
      tbase = vr.views[v].tile_base;
    }
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
    const int w = x1 - x0 + 1, area = w * (y1 - y0 + 1);
    const float4 p0 = pg0[g], p1 = pg1[g];
    const float relax = prelax[g];
    uint32_t o = offs[g];
    for (int base = 0; base < area; base += 256) {
      const int k = base + (int)threadIdx.x;
      const int tx = x0 + k % w, ty = y0 + k / w;
      bool keep = k < area;
      if (FILTER && keep && relax < 0.25f) keep = tile_keep(p0, p1, relax, tx, ty, W, H);
      uint32_t tot;
      const uint32_t pos = o + block_excl_scan256(keep ? 1u : 0u, s_scan, &tot);
      if (keep && pos < cap) {
        const uint32_t t = tbase + (uint32_t)(ty * tiles_x + tx);
        tkey[pos] = t | (kWholeTileBox << 16);
        tval[pos] = g;
        atomicAdd(&s_hist[0][t & m0], 1u);
        atomicAdd(&s_hist[1][(t >> bits0) & 255u], 1u);
      }
      o += tot;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 512; i += blockDim.x) {
    const uint32_t v = (&s_hist[0][0])[i];
    if (v) atomicAdd(hist + 4 * 256 + i, v);
  }
}

__global__ __launch_bounds__(256) void tile_ranges(const uint32_t* __restrict__ key, const uint32_t* ctr,
                                                   uint2* __restrict__ ranges, uint32_t ntiles) {
  const uint32_t n = ctr[C_NPAIRS];
  const uint32_t nq = (n + 3u) / 4u;
  // four consecutive keys per thread with one 16-byte load, and the keys on
  // either side of them: one memory latency per thread
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    const uint32_t i0 = 4u * q;
    uint32_t k[6];
    if (i0 + 4u <= n) {
      const uint4 v = reinterpret_cast<const uint4*>(key)[q];
      k[1] = v.x;
      k[2] = v.y;
      k[3] = v.z;
      k[4] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < n ? key[i0 + j] : 0u;
    }
    k[0] = i0 > 0 ? key[i0 - 1u] : 0u;
    k[5] = i0 + 4u < n ? key[i0 + 4u] : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t i = i0 + j;
      if (i >= n) break;
      const uint32_t t = k[1 + j] & 0xFFFFu;   // the tile id (the pixel box above it)
      if (t >= ntiles) continue;
      if (i == 0 || (k[j] & 0xFFFFu) != t) ranges[t].x = i;
      if (i + 1 == n || (k[2 + j] & 0xFFFFu) != t) ranges[t].y = i + 1;
    }
  }
}

// ---------------------------------------------------------------- blend ----
//
// Front-to-back blending (Eq. 3) per pixel, over the tile's pairs in depth
// order. Canonical arithmetic: the depth axis is cut into fixed bins (the top
// bits of the float32 depth: sixteen bins per octave); within a bin a pixel
// accumulates C_b = sum alpha T_b c and T_b = prod (1 - alpha) starting from
// (0, 1), and bins are combined in order, C = C + T C_b, T = T T_b. Blending
// stops before the first Gaussian whose blend would take the global
// transmittance T * T_b below 1e-4. Because the bins are a property of each
// Gaussian, this arithmetic is the same whether a tile is blended by one
// workgroup or split over several, and the same with and without the
// preemptive filter (whose pair lists are subsequences of the plain ones).
//
// When asked for, tiles with more than split_min pairs are split into jobs of
// whole bins; each job
// writes per-bin (C_b, T_b) per pixel and a composite pass combines them,
// re-blending exactly the one bin in which a pixel's transmittance crosses
// 1e-4.
//
// Within a job, each wave owns one 16x4 band of the tile; every batch of 256
// Gaussians is staged in LDS with, per band, the ordered list of those whose
// pixel box (half-extents in pg2.w, beyond which no pixel is blended) reaches
// it.
constexpr uint32_t kTierMin[3] = {16384, 4096, 1024};   // tiles blended first, heaviest tier first
// Workgroups whose waves blend the two heaviest tiers band by band, for the two
// layouts of vy_render_opts.band_jobs. Latency: jobs are halves of bands (8x4
// pixels) on 320 workgroups; the horizon's Gaussians are a few pixels wide, so
// half a band sees about two thirds of the band's entries and the longest job
// (one frame's critical path) walks correspondingly fewer. Throughput: whole
// bands on 128 workgroups, which spends less work in all (each job scans its
// tile's list once per band rather than once per half) and leaves more of the
// chip to the tile jobs of frames that overlap.
constexpr int kBandWGsLatency = 320;
constexpr int kBandWGsThroughput = 128;
constexpr int kMaxBins = 256;
constexpr uint32_t kMaxHeavy = 2048;
constexpr uint32_t kMaxJobsPerTile = 64;
constexpr uint32_t kMaxBinSlots = 32768;
constexpr int kHeavyRec = 4 + (kMaxBins + 1) + kMaxBins;   // tile, nb, slot base, -, pos[nb+1], key[nb]

VY_DEV uint32_t depth_bin(float z) { return __float_as_uint(z) >> 19; }

// Pixel rule of the blend: Gaussian i is evaluated at pixel centre f only when
// |mean2d - f| <= (rx, ry) per axis, the half-extents of its pixel box, with
// the differences computed exactly as for rho. Outside the box alpha < alpha*
// (and with the filter, Eq. 4 fails), so the rule removes only evaluations
// that cannot blend; stating it explicitly makes every walk of a tile list
// (per band, per pixel, split by depth) evaluate the same (Gaussian, pixel)
// pairs bit for bit.
//
// Can the pixel box (half-extents packed in `ext` as rx | ry << 16) hold a
// pixel centre of the band starting at (xa, ya), `xw` + 1 pixels wide (16, or
// 8 for half a band) and 4 high? A half-pixel slack makes this a superset of
// the pixel rule under rounding.
VY_DEV bool band_hit(float mx, float my, float ext, float xa, float ya, float xw = 15.f) {
  const uint32_t e = __float_as_uint(ext);
  const float rx = (float)(e & 0xFFFFu) + 0.5f, ry = (float)(e >> 16) + 0.5f;
  return (mx + rx >= xa) && (mx - rx <= xa + xw) && (my + ry >= ya) && (my - ry <= ya + 3.f);
}

// LDS staging of pairs [b0, min(b0 + 256, pe)) of a tile: per band, the
// ordered list of (depth bin << 8 | batch index) of the entries whose pixel box
// may reach it, and their records in the same order (r0 = pg0, r1 = pg1 with
// ry in .w, r2 = pg2 with rx in .w: the pixel box half-extents as floats in
// place of the depth and the packed extents), so that a band reads an entry's
// key and record with independent LDS loads. Returns this wave's list length.
struct Stage {
  float4 r0[4][256], r1[4][256], r2[4][256];   // records per band, in band-list order
  uint32_t list[4][256];   // (depth bin << 8) | batch index, in depth order
  uint32_t wc[4][4];
};

VY_DEV int stage_batch(Stage& S, uint32_t b0, uint32_t pe, const uint32_t* __restrict__ tval,
                       const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                       const float4* __restrict__ pg2, uint32_t n_g, int tx, int ty) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const uint32_t idx = b0 + threadIdx.x;
  uint32_t qm = 0, key = 0;
  float4 a, b1, c1;
  if (idx < pe) {
    uint32_t g = tval[idx];
    if (g >= n_g) g = 0;
    a = pg0[g];
    const float4 b = pg1[g], c = pg2[g];
    const uint32_t ex = __float_as_uint(c.w);
    b1 = make_float4(b.x, b.y, b.z, (float)(ex >> 16));      // .w = ry
    c1 = make_float4(c.x, c.y, c.z, (float)(ex & 0xFFFFu));  // .w = rx
    key = depth_bin(b.w);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      qm |= band_hit(a.x, a.y, c.w, tx * kTileSize + 0.5f, ty * kTileSize + q * 4 + 0.5f) ? (1u << q) : 0u;
  }
  uint64_t bal[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bal[q] = __ballot((qm >> q) & 1u);
    if (l == 0) S.wc[q][w] = (uint32_t)__popcll(bal[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if ((qm >> q) & 1u) {
      uint32_t base = 0;
      for (int ww = 0; ww < w; ++ww) base += S.wc[q][ww];
      const uint32_t pos = base + (uint32_t)__popcll(bal[q] & lanemask_lt());
      S.list[q][pos] = (key << 8) | threadIdx.x;
      S.r0[q][pos] = a;
      S.r1[q][pos] = b1;
      S.r2[q][pos] = c1;
    }
  }
  __syncthreads();
  return (int)(S.wc[w][0] + S.wc[w][1] + S.wc[w][2] + S.wc[w][3]);
}

// Tile planning. Tiles with more than split_min pairs are split into jobs
// (tile_flag = heavy index + 2); other tiles with many pairs are queued in
// three tiers by size (tile_flag = 1) and blended first, heaviest tier first,
// so that the longest tiles start at once; the rest (tile_flag = 0) follow in
// tile order.
__global__ __launch_bounds__(256) void plan_tiles(const uint2* __restrict__ ranges, int ntiles,
                                                  uint32_t* __restrict__ tile_flag, uint32_t* __restrict__ heavy_list,
                                                  uint32_t* __restrict__ tiers, uint32_t* ctr, uint32_t split_min) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y > r.x ? r.y - r.x : 0u;
    uint32_t f = 0;
    if (len > split_min) {
      const uint32_t h = fetch_add(ctr + C_NHEAVY, 1u);
      if (h < kMaxHeavy) {
        heavy_list[h] = (uint32_t)t;
        f = h + 2;
      }
    }
    // the tier (the first threshold the tile's list exceeds), appended with
    // one atomic per wave and tier (the order within a tier does not matter)
    int tier = -1;
    if (f == 0)
      for (int k = 2; k >= 0; --k)
        if (len > kTierMin[k]) tier = k;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint64_t bal = __ballot(tier == k);
      if (bal == 0ull) continue;
      const int leader = __builtin_ctzll(bal);
      uint32_t slot0 = 0;
      if ((int)lane() == leader) slot0 = fetch_add(ctr + C_NTIER + k, (uint32_t)__popcll(bal));
      slot0 = (uint32_t)__shfl((int)slot0, leader, 64);
      if (tier == k) tiers[(size_t)k * ntiles + slot0 + (uint32_t)__popcll(bal & lanemask_lt())] = (uint32_t)t;
    }
    if (tier >= 0) f = 1;
    tile_flag[t] = f;
  }
}

// One workgroup per heavy tile: find its depth-bin boundaries (in order, by a
// block scan over the tile's pairs) and cut it into jobs of whole bins of
// about len/48 pairs (at least split_min/2) each.
__global__ __launch_bounds__(256) void plan_heavy(const uint2* __restrict__ ranges,
                                                  const uint32_t* __restrict__ tval,
                                                  const float4* __restrict__ pg1,
                                                  const uint32_t* __restrict__ heavy_list,
                                                  uint32_t* __restrict__ tile_flag, uint32_t* __restrict__ heavy_rec,
                                                  uint4* __restrict__ jobs, uint32_t* __restrict__ slot_owner,
                                                  uint32_t* ctr, uint32_t n_g, uint32_t split_min) {
  __shared__ uint32_t s_pos[kMaxBins + 1], s_key[kMaxBins], s_scan[8], s_base, s_ok;
  uint32_t nh = ctr[C_NHEAVY];
  if (nh > kMaxHeavy) nh = kMaxHeavy;
  for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const uint32_t tile = heavy_list[h];
    const uint2 r = ranges[tile];
    uint32_t nb = 0;   // uniform
    for (uint32_t c0 = r.x; c0 < r.y; c0 += blockDim.x) {
      const uint32_t i = c0 + threadIdx.x;
      uint32_t k = 0, kp = 0;
      bool bnd = false;
      if (i < r.y) {
        const uint32_t g = tval[i];
        k = g < n_g ? depth_bin(pg1[g].w) : 0u;
        if (i == r.x) {
          bnd = true;
        } else {
          const uint32_t gp = tval[i - 1];
          kp = gp < n_g ? depth_bin(pg1[gp].w) : 0u;
          bnd = k != kp;
        }
      }
      uint32_t tot;
      const uint32_t o = nb + block_excl_scan256(bnd ? 1u : 0u, s_scan, &tot);
      if (bnd && o < (uint32_t)kMaxBins) {
        s_pos[o] = i;
        s_key[o] = k;
      }
      nb += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t ok = nb <= (uint32_t)kMaxBins ? 1u : 0u;
      if (ok) {
        s_pos[nb] = r.y;
        const uint32_t base = fetch_add(ctr + C_SLOTS, nb);
        if (base + nb > kMaxBinSlots) ok = 0;
        s_base = base;
      }
      s_ok = ok;
    }
    __syncthreads();
    uint32_t* rec = heavy_rec + (size_t)h * kHeavyRec;
    if (s_ok) {
      for (uint32_t a = threadIdx.x; a <= nb; a += blockDim.x) rec[4 + a] = s_pos[a];
      for (uint32_t a = threadIdx.x; a < nb; a += blockDim.x) {
        rec[4 + kMaxBins + 1 + a] = s_key[a];
        slot_owner[s_base + a] = h;
      }
      if (threadIdx.x == 0) {
        rec[0] = tile;
        rec[1] = nb;
        rec[2] = s_base;
        const uint32_t len = r.y - r.x;
        uint32_t ch = len / 48;
        if (ch < split_min / 2) ch = split_min / 2;
        uint32_t j0 = 0, nj = 0;
        while (j0 < nb) {
          uint32_t j1 = j0 + 1;
          while (j1 < nb && (s_pos[j1] - s_pos[j0] < ch || nj + 1 >= kMaxJobsPerTile)) ++j1;
          const uint32_t jid = fetch_add(ctr + C_NJOBS, 1u);
          if (jid < kMaxHeavy * kMaxJobsPerTile) jobs[jid] = make_uint4(h, j0, j1, 0u);
          ++nj;
          j0 = j1;
        }
      }
    } else if (threadIdx.x == 0) {
      tile_flag[tile] = 0;   // blend it in one piece (with the other tiles)
    }
    __syncthreads();
  }
}

// The exponential of alpha = min(0.99, theta e^rho) (Eq. 3): the hardware
// exponential, or (LUT) the lookup table of Section 4.2: m + 1 values
// e^(-5.55 k / m), k = 0..m, over the effective range [-5.55, 0] of rho, read
// at the nearest node, index round(rho / -5.55 * m) (clamped to m; alpha is
// below alpha* there for theta <= 1). The table lives in LDS.
constexpr int kTransposedMax = 4;   // live pixels of a band at most for the entry-parallel walk
constexpr int kLutMax = 128;
constexpr double kLutRange = 5.55;
struct ExpLut {
  const float* tab;
  float scale;   // m / 5.55
  int m;
};

template <bool LUT>
VY_DEV float exp_rho(float power, const ExpLut& L) {
  if (!LUT) return __expf(power);
  const int k = (int)rintf(-power * L.scale);
  return L.tab[k < L.m ? k : L.m];
}

// Per-pixel blending state of one job.
struct PixAcc {
  float Tt, C0, C1, C2;     // combined over finished bins (one-piece mode)
  float Tb, Cb0, Cb1, Cb2;  // current bin
  int32_t nt, nb;
  uint32_t stop_pos;        // tile-list position of the Gaussian where blending stopped (save mode)
  uint32_t last;            // tile-list position of the last blended Gaussian (save mode)
  bool done;
  uint32_t cur_key;         // depth bin of the current bin (0xFFFFFFFF before the first)
  uint32_t lb;              // local index of the current bin (split mode)
};

struct SplitOut {           // where split-mode jobs write their per-bin results
  float4* bin_c;
  int32_t* bin_n;
  const uint32_t* bkey;     // keys of the job's bins (heavy record), bkey[lb - lbin0]
  uint32_t slot_base, lbin0, lbin1;
  int pix;
};

VY_DEV void put_bin(const SplitOut& o, uint32_t lb, float4 v, int32_t n) {
  const size_t k = ((size_t)(o.slot_base + lb)) * 256 + o.pix;
  o.bin_c[k] = v;
  o.bin_n[k] = n;
}

// Blend pairs [pb, pe) of tile (tx, ty) into A. SPLIT: per-bin results go to
// `so` and a pixel stops only when its own bin's T falls below 1e-4 (marking
// the bin with T = 0 for the composite); otherwise bins are combined in place
// and a pixel stops before the Gaussian that would take Tt * T_b below 1e-4.
// A pixel enters depth bin `key`: close its current bin (combine it in place,
// or write it out in split mode, together with any bins it skipped).
template <bool SPLIT>
VY_DEV void bin_enter(PixAcc& A, uint32_t key, const SplitOut& so) {
  if (SPLIT) {
    if (A.cur_key != 0xFFFFFFFFu) {
      put_bin(so, A.lb, make_float4(A.Cb0, A.Cb1, A.Cb2, A.Tb), A.nb);
      ++A.lb;
    }
    while (A.lb < so.lbin1 && so.bkey[A.lb - so.lbin0] != key) {   // bins with nothing for this pixel
      put_bin(so, A.lb, make_float4(0.f, 0.f, 0.f, 1.f), 0);
      ++A.lb;
    }
  } else {
    A.C0 = fmaf(A.Tt, A.Cb0, A.C0);
    A.C1 = fmaf(A.Tt, A.Cb1, A.C1);
    A.C2 = fmaf(A.Tt, A.Cb2, A.C2);
    A.Tt = A.Tt * A.Tb;
    A.nt += A.nb;
  }
  A.Tb = 1.f;
  A.Cb0 = A.Cb1 = A.Cb2 = 0.f;
  A.nb = 0;
}

// One Gaussian of the band list for every pixel of the wave (slow path of
// blend_range, used around depth-bin boundaries): alpha = min(0.99, theta e^rho)
// (Eq. 3), skipped below alpha* (with the filter, decided before the
// exponential by Eq. 4); blending stops before a Gaussian that would take the
// transmittance (Tt * T_b, or T_b alone in split mode) below 1e-4.
template <bool FILTER, bool SPLIT, bool SAVE, bool LUT>
VY_DEV void blend_one(uint32_t key, const float4 p0, const float4 p1, const float4 p2, float fxp, float fyp,
                      PixAcc& A, const SplitOut& so, uint32_t pos, const ExpLut& L) {
  if (key != A.cur_key) {                 // a new depth bin begins (wave-uniform)
    if (!A.done) bin_enter<SPLIT>(A, key, so);   // a finished pixel keeps its state frozen
    A.cur_key = key;
  }
  const float dx = p0.x - fxp, dy = p0.y - fyp;
  // rho = A dx^2 + B dx dy + C dy^2, clamped to <= 0
  float power = fmaf(dx, fmaf(p0.z, dx, p0.w * dy), (p1.x * dy) * dy);
  power = fminf(power, 0.f);
  bool live = !A.done && fabsf(dx) <= p2.w && fabsf(dy) <= p1.w;   // pixel rule
  if (FILTER) live = live && power >= p1.z;   // Eq. 4: rho < log(alpha*) - log(theta) => skip
  if (__ballot(live) == 0ull) return;        // the exponential is needed by no pixel of the band
  const float alpha = fminf(kAlphaMax, p1.y * exp_rho<LUT>(power, L));
  const bool ok = live && alpha >= kAlphaMin;
  const float Tn = A.Tb * (1.f - alpha);
  const bool stop = ok && (SPLIT ? (Tn < kTMin) : (A.Tt * Tn < kTMin));
  const bool bl = ok && !stop;
  const float wgt = bl ? alpha * A.Tb : 0.f;
  A.Cb0 = fmaf(wgt, p2.x, A.Cb0);
  A.Cb1 = fmaf(wgt, p2.y, A.Cb1);
  A.Cb2 = fmaf(wgt, p2.z, A.Cb2);
  A.Tb = bl ? Tn : ((SPLIT && stop) ? 0.f : A.Tb);
  A.nb += bl ? 1 : 0;
  if (SAVE && bl) A.last = pos;
  if (SAVE && stop) A.stop_pos = pos;
  A.done = A.done || stop;
}

// Per-pixel walk of up to 64 band-list entries [jj, jj + m) (one-piece mode):
// each lane visits, in list order, only the entries that pass the pixel rule
// at its own pixel centre (bits of `mk`). The depth bins that the skipped
// entries would have opened and left empty fold as exact no-ops (C + T 0 = C,
// T 1 = T), so the result is bitwise that of the band walk.
template <bool FILTER, bool SAVE, bool LUT>
VY_DEV void blend_sparse(const Stage& S, int w, int jj, uint64_t mk, uint32_t b0, float fxp, float fyp, PixAcc& A,
                         const ExpLut& L) {
  // Up to four of the lane's entries per step: their records are loaded and
  // their alphas computed independently; only the transmittance chain is
  // sequential. A depth bin is opened lazily, at the first entry that blends
  // in it: nothing changes the pixel's state in between, so the fold is the
  // same as at the bin's first entry.
  while (__ballot(mk != 0ull) != 0ull) {
    int pos[4];
    bool vk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vk[u] = mk != 0ull;
      pos[u] = jj + (vk[u] ? __builtin_ctzll(mk) : 0);
      mk &= mk - 1ull;
    }
    uint32_t e[4];
    float4 p0[4], p1[4], p2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      e[u] = S.list[w][pos[u]];
      p0[u] = S.r0[w][pos[u]];
      p1[u] = S.r1[w][pos[u]];
      p2[u] = S.r2[w][pos[u]];
    }
    float al[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float dx = p0[u].x - fxp, dy = p0[u].y - fyp;
      const float power = fminf(fmaf(dx, fmaf(p0[u].z, dx, p0[u].w * dy), (p1[u].x * dy) * dy), 0.f);
      bool o = vk[u];
      if (FILTER) o = o & (power >= p1[u].z);   // Eq. 4 before the exponential
      al[u] = fminf(kAlphaMax, p1[u].y * exp_rho<LUT>(power, L));
      ok[u] = o & (al[u] >= kAlphaMin);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u] || A.done) continue;
      const uint32_t key = e[u] >> 8;
      if (key != A.cur_key) {
        A.C0 = fmaf(A.Tt, A.Cb0, A.C0);
        A.C1 = fmaf(A.Tt, A.Cb1, A.C1);
        A.C2 = fmaf(A.Tt, A.Cb2, A.C2);
        A.Tt = A.Tt * A.Tb;
        A.nt += A.nb;
        A.Tb = 1.f;
        A.Cb0 = A.Cb1 = A.Cb2 = 0.f;
        A.nb = 0;
        A.cur_key = key;
      }
      // the stop is taken by selects, not a branch: a stopping lane adds
      // 0 * colour (+0, colours are >= 0), so its sums are unchanged bitwise
      const float Tn = A.Tb * (1.f - al[u]);
      const bool stop = A.Tt * Tn < kTMin;
      const float wgt = stop ? 0.f : al[u] * A.Tb;
      A.Cb0 = fmaf(wgt, p2[u].x, A.Cb0);
      A.Cb1 = fmaf(wgt, p2[u].y, A.Cb1);
      A.Cb2 = fmaf(wgt, p2[u].z, A.Cb2);
      A.Tb = stop ? A.Tb : Tn;
      A.nb += stop ? 0 : 1;
      if (SAVE) {
        A.last = stop ? A.last : b0 + (e[u] & 255u);
        A.stop_pos = stop ? b0 + (e[u] & 255u) : A.stop_pos;
      }
      A.done = stop;
    }
    if (A.done) mk = 0ull;
  }
}

// Few pixels of the band still blend (the tail of a long list, where most
// pixels have stopped): each such pixel in turn, the lanes evaluate the
// chunk's entries [jj, jj + m) at that pixel in parallel, one entry per lane
// (pixel rule, rho, Eq. 4, alpha: the float operations of the per-pixel walk),
// and the pixel's sequential blend then runs over the entries that pass, in
// list order, on wave-uniform copies of its state (the same operations in the
// same order as blend_sparse: bitwise the same result).
VY_DEV float rl(float v, int k) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k)); }
VY_DEV uint32_t rl(uint32_t v, int k) { return (uint32_t)__builtin_amdgcn_readlane((int)v, k); }
VY_DEV int32_t rl(int32_t v, int k) { return __builtin_amdgcn_readlane(v, k); }

template <bool FILTER, bool SAVE, bool LUT>
VY_DEV void blend_transposed(const Stage& S, int w, int jj, int m, uint32_t b0, float fxp, float fyp, PixAcc& A,
                             const ExpLut& L) {
  const int l = (int)(threadIdx.x & 63);
  float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
  uint32_t e = 0;
  if (l < m) {
    e = S.list[w][jj + l];
    q0 = S.r0[w][jj + l];
    q1 = S.r1[w][jj + l];
    q2 = S.r2[w][jj + l];
  }
  uint64_t alive = __ballot(!A.done);
  while (alive) {
    const int p = __builtin_ctzll(alive);
    alive &= alive - 1ull;
    const float fx = rl(fxp, p), fy = rl(fyp, p);
    bool ok = false;
    float al = 0.f;
    if (l < m) {
      const float dx = q0.x - fx, dy = q0.y - fy;
      const bool cov = fabsf(dx) <= q2.w && fabsf(dy) <= q1.w;   // the pixel rule
      const float power = fminf(fmaf(dx, fmaf(q0.z, dx, q0.w * dy), (q1.x * dy) * dy), 0.f);
      bool o = cov;
      if (FILTER) o = o & (power >= q1.z);                       // Eq. 4 before the exponential
      al = fminf(kAlphaMax, q1.y * exp_rho<LUT>(power, L));
      ok = o & (al >= kAlphaMin);
    }
    uint64_t okm = __ballot(ok);
    // pixel p's state, the same in every lane
    float Tt = rl(A.Tt, p), C0 = rl(A.C0, p), C1 = rl(A.C1, p), C2 = rl(A.C2, p);
    float Tb = rl(A.Tb, p), Cb0 = rl(A.Cb0, p), Cb1 = rl(A.Cb1, p), Cb2 = rl(A.Cb2, p);
    int32_t nt = rl(A.nt, p), nb = rl(A.nb, p);
    uint32_t stop_pos = rl(A.stop_pos, p), last = rl(A.last, p), cur_key = rl(A.cur_key, p);
    bool done = false;
    while (okm) {
      const int k = __builtin_ctzll(okm);
      okm &= okm - 1ull;
      const float a = rl(al, k);
      const uint32_t ek = rl(e, k);
      const float4 c = S.r2[w][jj + k];
      const uint32_t key = ek >> 8;
      if (key != cur_key) {
        C0 = fmaf(Tt, Cb0, C0);
        C1 = fmaf(Tt, Cb1, C1);
        C2 = fmaf(Tt, Cb2, C2);
        Tt = Tt * Tb;
        nt += nb;
        Tb = 1.f;
        Cb0 = Cb1 = Cb2 = 0.f;
        nb = 0;
        cur_key = key;
      }
      const float Tn = Tb * (1.f - a);
      const bool stop = Tt * Tn < kTMin;
      const float wgt = stop ? 0.f : a * Tb;
      Cb0 = fmaf(wgt, c.x, Cb0);
      Cb1 = fmaf(wgt, c.y, Cb1);
      Cb2 = fmaf(wgt, c.z, Cb2);
      Tb = stop ? Tb : Tn;
      nb += stop ? 0 : 1;
      if (SAVE) {
        last = stop ? last : b0 + (ek & 255u);
        stop_pos = stop ? b0 + (ek & 255u) : stop_pos;
      }
      if (stop) {
        done = true;
        break;
      }
    }
    if (l == p) {
      A.Tt = Tt;
      A.C0 = C0;
      A.C1 = C1;
      A.C2 = C2;
      A.Tb = Tb;
      A.Cb0 = Cb0;
      A.Cb1 = Cb1;
      A.Cb2 = Cb2;
      A.nt = nt;
      A.nb = nb;
      A.stop_pos = stop_pos;
      A.last = last;
      A.cur_key = cur_key;
      A.done = done;
    }
  }
}

// Coverage masks of band-list entries [jj, jj + m) for the wave's pixels: bit
// k of lane (c, r) is set when entry jj + k passes the pixel rule at the pixel
// centre (xa + c, ya + r).
VY_DEV uint64_t cover_masks(const Stage& S, int w, int jj, int m, float xa, float ya, int l) {
  float mx = 0.f, my = 0.f, rx = -1.f, ry = -1.f;   // empty box for lanes past the chunk
  if (l < m) {
    const float4 a = S.r0[w][jj + l];
    mx = a.x;
    my = a.y;
    rx = S.r2[w][jj + l].w;
    ry = S.r1[w][jj + l].w;
  }
  const int c = l & 15, r = l >> 4;
  uint64_t mc = 0ull, mr = 0ull;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float f = xa + (float)i;   // the pixel centre, exactly as the blend forms it
    const uint64_t b = __ballot(fabsf(mx - f) <= rx);
    mc = c == i ? b : mc;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float f = ya + (float)i;
    const uint64_t b = __ballot(fabsf(my - f) <= ry);
    mr = r == i ? b : mr;
  }
  return mc & mr;
}

// Blend band-list entries [jc, jc + mc) (mc <= 64) of the wave's LDS region
// w, tile-list positions counted from b0, for the band whose first pixel
// centre is (xa, ya). walk 0 (automatic) and 2: per pixel, each lane over its
// own entries, and (walk 0) entry-parallel once at most kTransposedMax pixels
// are live; walk 1, and split jobs: all pixels together. (On the full-scale
// walkthrough the per-pixel walk measured faster than the together walk also
// on chunks whose busiest pixel covers most of the entries.)
template <bool FILTER, bool SPLIT, bool SAVE, bool LUT>
VY_DEV void walk_chunk(const Stage& S, int w, int jc, int mc, uint32_t b0, float xa, float ya, float fxp, float fyp,
                       PixAcc& A, const SplitOut& so, int walk, const ExpLut& L) {
  if (!SPLIT && walk != 1) {
    const uint64_t live = __ballot(!A.done);
    if (live == 0ull) return;
    // the tail of a long list, where few pixels still blend: entry-parallel walk per pixel
    if (walk == 0 && __popcll(live) <= kTransposedMax) {
      blend_transposed<FILTER, SAVE, LUT>(S, w, jc, mc, b0, fxp, fyp, A, L);
      return;
    }
    uint64_t mk = cover_masks(S, w, jc, mc, xa, ya, (int)(threadIdx.x & 63));
    if (A.done) mk = 0ull;
    blend_sparse<FILTER, SAVE, LUT>(S, w, jc, mk, b0, fxp, fyp, A, L);
    return;
  }
  for (int jj = jc; jj < jc + mc; jj += 4) {
    if (__ballot(!A.done) == 0ull) return;   // the whole band has terminated
    const uint4 e4 = *reinterpret_cast<const uint4*>(&S.list[w][jj]);
    const int m = jc + mc - jj < 4 ? jc + mc - jj : 4;
    const uint32_t e[4] = {(uint32_t)__builtin_amdgcn_readfirstlane(e4.x),
                           (uint32_t)__builtin_amdgcn_readfirstlane(e4.y),
                           (uint32_t)__builtin_amdgcn_readfirstlane(e4.z),
                           (uint32_t)__builtin_amdgcn_readfirstlane(e4.w)};
    float4 q0[4], q1[4], q2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int pos = k < m ? jj + k : jj;
      q0[k] = S.r0[w][pos];
      q1[k] = S.r1[w][pos];
      q2[k] = S.r2[w][pos];
    }
    const uint32_t key = e[0] >> 8;
    if (m == 4 && key == A.cur_key && (e[1] >> 8) == key && (e[2] >> 8) == key && (e[3] >> 8) == key) {
      // fast path, one depth bin: rho and the alphas are independent of each
      // other; only the transmittance chain below is sequential
      float pw[4];
      bool lv[4];
      bool any = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float dx = q0[k].x - fxp, dy = q0[k].y - fyp;
        pw[k] = fminf(fmaf(dx, fmaf(q0[k].z, dx, q0[k].w * dy), (q1[k].x * dy) * dy), 0.f);
        lv[k] = !A.done && fabsf(dx) <= q2[k].w && fabsf(dy) <= q1[k].w;   // pixel rule
        if (FILTER) lv[k] = lv[k] && pw[k] >= q1[k].z;   // Eq. 4 before the exponential
        any = any || lv[k];
      }
      if (__ballot(any) == 0ull) continue;   // no pixel of the band needs these four
      float al[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) al[k] = fminf(kAlphaMax, q1[k].y * exp_rho<LUT>(pw[k], L));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool okk = lv[k] && al[k] >= kAlphaMin && !A.done;
        const float Tn = A.Tb * (1.f - al[k]);
        const bool stop = okk && (SPLIT ? (Tn < kTMin) : (A.Tt * Tn < kTMin));
        const bool bl = okk && !stop;
        const float wgt = bl ? al[k] * A.Tb : 0.f;
        A.Cb0 = fmaf(wgt, q2[k].x, A.Cb0);
        A.Cb1 = fmaf(wgt, q2[k].y, A.Cb1);
        A.Cb2 = fmaf(wgt, q2[k].z, A.Cb2);
        A.Tb = bl ? Tn : ((SPLIT && stop) ? 0.f : A.Tb);
        A.nb += bl ? 1 : 0;
        if (SAVE && bl) A.last = b0 + (e[k] & 255u);
        if (SAVE && stop) A.stop_pos = b0 + (e[k] & 255u);
        A.done = A.done || stop;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < m)
          blend_one<FILTER, SPLIT, SAVE, LUT>(e[k] >> 8, q0[k], q1[k], q2[k], fxp, fyp, A, so, b0 + (e[k] & 255u),
                                              L);
    }
  }
}

// Blend pairs [pb, pe) of tile (tx, ty) into A. SPLIT: per-bin results go to
// `so` and a pixel stops only when its own bin's T falls below 1e-4 (marking
// the bin with T = 0 for the composite); otherwise bins are combined in place.
// The band list is walked four entries at a time: all LDS loads are issued
// first, and when the four share the current depth bin their alphas are
// computed independently before the sequential transmittance chain, which
// keeps the per-Gaussian latency low on the tiles with the longest lists.
template <bool FILTER, bool SPLIT, bool SAVE, bool LUT>
VY_DEV void blend_range(Stage& S, uint32_t pb, uint32_t pe, const uint32_t* __restrict__ tval,
                        const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                        const float4* __restrict__ pg2, uint32_t n_g, int tx, int ty, float fxp, float fyp,
                        PixAcc& A, const SplitOut& so, int walk, const ExpLut& L) {
  const int w = threadIdx.x >> 6;
  for (uint32_t b0 = pb; b0 < pe; b0 += 256) {
    if (__syncthreads_count(A.done) == 256) break;
    const int cnt = stage_batch(S, b0, pe, tval, pg0, pg1, pg2, n_g, tx, ty);
    for (int jc = 0; jc < cnt; jc += 64) {
      if (__ballot(!A.done) == 0ull) break;
      walk_chunk<FILTER, SPLIT, SAVE, LUT>(S, w, jc, cnt - jc < 64 ? cnt - jc : 64, b0, tx * kTileSize + 0.5f,
                                           ty * kTileSize + w * 4 + 0.5f, fxp, fyp, A, so, walk, L);
    }
    __syncthreads();
  }
}

// Final fold of the open depth bin and the pixel's outputs (image with the
// background behind the remaining transmittance; in save mode T, the number of
// blended Gaussians, the number of tile-list entries walked and the tile-list
// position of the last blended Gaussian, -1 if none).
template <bool SAVE>
VY_DEV void pixel_out(PixAcc& A, const RCam& cam, int px, int py, uint32_t pb, uint32_t pe, float* __restrict__ img,
                      float* __restrict__ Tout, int32_t* __restrict__ Nout, int32_t* __restrict__ Eout,
                      int32_t* __restrict__ Lout) {
  A.C0 = fmaf(A.Tt, A.Cb0, A.C0);
  A.C1 = fmaf(A.Tt, A.Cb1, A.C1);
  A.C2 = fmaf(A.Tt, A.Cb2, A.C2);
  A.Tt = A.Tt * A.Tb;
  A.nt += A.nb;
  const size_t hw = (size_t)cam.W * cam.H, o = (size_t)py * cam.W + px;
  img[o] = fmaf(A.Tt, cam.bg[0], A.C0);
  img[hw + o] = fmaf(A.Tt, cam.bg[1], A.C1);
  img[2 * hw + o] = fmaf(A.Tt, cam.bg[2], A.C2);
  if (SAVE) {
    Tout[o] = A.Tt;
    Nout[o] = A.nt;
    Eout[o] = (int32_t)((A.stop_pos != 0xFFFFFFFFu ? A.stop_pos + 1u : pe) - pb);
    Lout[o] = A.last == 0xFFFFFFFFu ? -1 : (int32_t)A.last;
  }
}

VY_DEV void pix_init(PixAcc& A, bool inside) {
  A.Tt = 1.f;
  A.C0 = A.C1 = A.C2 = 0.f;
  A.Tb = 1.f;
  A.Cb0 = A.Cb1 = A.Cb2 = 0.f;
  A.nt = A.nb = 0;
  A.stop_pos = 0xFFFFFFFFu;
  A.last = 0xFFFFFFFFu;
  A.done = !inside;
  A.cur_key = 0xFFFFFFFFu;
  A.lb = 0;
}

// Wave-level blend of one 16x4 band of a heavy tile (or, for half >= 0, of
// its left or right 8x4 half: the lanes of the other half start as finished
// pixels and entries are kept for the half's pixels only, which changes no
// pixel's result), with no workgroup barriers, so that the bands of a tile
// finish independently: the wave walks
// the tile's pairs in chunks of 64 * kBandParts (kBandParts per lane) with the
// records of the next chunk and the cut positions of the one after in flight, compacts the entries
// whose pixel box may reach the band into its LDS region, and blends them as
// the workgroup walk does (same rules, bitwise the same pixels).
constexpr int kBandParts = 4;   // a band job stages 64 * kBandParts pairs per step (at most 256: its LDS list)
static_assert(kBandParts >= 1 && kBandParts <= 4, "the band list holds 256 entries");

template <bool FILTER, bool SAVE, bool LUT>
VY_DEV void blend_band(Stage& S, int w, int tx, int ty, int band, int half, uint32_t pb, uint32_t pe,
                       const uint32_t* __restrict__ tval, const float4* __restrict__ pg0,
                       const float4* __restrict__ pg1, const float4* __restrict__ pg2,
                       const float* __restrict__ prelax, uint32_t n_g, const RCam& cam,
                       float* __restrict__ img, float* __restrict__ Tout, int32_t* __restrict__ Nout,
                       int32_t* __restrict__ Eout, int32_t* __restrict__ Lout, int walk, const ExpLut& L) {
  const int l = (int)(threadIdx.x & 63);
  const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + band * 4 + (l >> 4);
  const bool inside = px < cam.W && py < cam.H && (half < 0 || (l & 15) >> 3 == half);
  PixAcc A;
  pix_init(A, inside);
  const SplitOut so{};
  const float fxp = px + 0.5f, fyp = py + 0.5f;
  const float xa = tx * kTileSize + 0.5f, ya = ty * kTileSize + band * 4 + 0.5f;
  const float xh = half > 0 ? xa + 8.f : xa, xw = half < 0 ? 15.f : 7.f;   // the pixels this job blends
  // chunks of kBandParts x 64 pairs: lane l holds pairs b0 + h * 64 + l; the
  // records of the next chunk and the cut positions of the one after are in
  // flight while a chunk is blended
  constexpr int NP = kBandParts, CH = 64 * kBandParts;
  float4 na[NP], nb[NP], nc[NP];
  float nr[NP];   // rounding allowances of rho (filter only)
  uint32_t g1[NP];
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    na[h] = nb[h] = nc[h] = make_float4(0.f, 0.f, 0.f, 0.f);
    nr[h] = 1.f;
    g1[h] = 0u;
    const uint32_t p0 = pb + h * 64 + l;
    if (p0 < pe) {
      uint32_t g = tval[p0];
      if (g >= n_g) g = 0;
      na[h] = pg0[g];
      nb[h] = pg1[g];
      nc[h] = pg2[g];
      if (FILTER) nr[h] = prelax[g];
    }
    const uint32_t p1 = pb + CH + h * 64 + l;
    if (p1 < pe) {
      g1[h] = tval[p1];
      if (g1[h] >= n_g) g1[h] = 0;
    }
  }
  for (uint32_t b0 = pb; b0 < pe; b0 += CH) {
    if (__ballot(!A.done) == 0ull) break;
    bool hit[NP];
    float4 a[NP], b[NP], c[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      a[h] = na[h];
      b[h] = nb[h];
      c[h] = nc[h];
      hit[h] = b0 + h * 64 + l < pe && band_hit(a[h].x, a[h].y, c[h].w, xh, ya, xw);
      // with the filter, Eq. 4 over the job's pixel centres as for tiles: an
      // entry whose rho stays below the threshold at every one of them fails
      // the per-pixel test everywhere, so dropping it changes no pixel; the
      // test runs here once per entry, in parallel over the lanes, instead of
      // once per entry of the sequential walk
      if (FILTER && hit[h] && nr[h] < 0.25f)
        hit[h] = rect_rho_max(a[h].x, a[h].y, a[h].z, a[h].w, b[h].x, xh, ya, xh + xw, ya + 3.f) * (1.f - nr[h]) >=
                 b[h].z;
    }
#pragma unroll
    for (int h = 0; h < NP; ++h) {   // records of the next chunk, cut positions of the one after
      if (b0 + CH + h * 64 + l < pe) {
        na[h] = pg0[g1[h]];
        nb[h] = pg1[g1[h]];
        nc[h] = pg2[g1[h]];
        if (FILTER) nr[h] = prelax[g1[h]];
      }
      if (b0 + 2 * CH + h * 64 + l < pe) {
        g1[h] = tval[b0 + 2 * CH + h * 64 + l];
        if (g1[h] >= n_g) g1[h] = 0;
      }
    }
    uint32_t base = 0;
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      const uint64_t bal = __ballot(hit[h]);
      if (hit[h]) {
        const uint32_t pos = base + (uint32_t)__popcll(bal & lanemask_lt());
        const uint32_t ex = __float_as_uint(c[h].w);
        S.list[w][pos] = (depth_bin(b[h].w) << 8) | (uint32_t)(h * 64 + l);
        S.r0[w][pos] = a[h];
        S.r1[w][pos] = make_float4(b[h].x, b[h].y, b[h].z, (float)(ex >> 16));
        S.r2[w][pos] = make_float4(c[h].x, c[h].y, c[h].z, (float)(ex & 0xFFFFu));
      }
      base += (uint32_t)__popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int cnt = (int)base;
    for (int jc = 0; jc < cnt; jc += 64) {
      if (__ballot(!A.done) == 0ull) break;
      walk_chunk<FILTER, false, SAVE, LUT>(S, w, jc, cnt - jc < 64 ? cnt - jc : 64, b0, xa, ya, fxp, fyp, A, so, walk,
                                           L);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (inside) pixel_out<SAVE>(A, cam, px, py, pb, pe, img, Tout, Nout, Eout, Lout);
}

// Band job over candidate batches (with the filter, without saved state).
// The sorted tile keys carry each pair's pixel box within its tile, so the
// wave first scans keys and cut positions, coalesced and two bulks of 256
// ahead, for the pairs whose box meets the job's pixels, and gathers the
// random 48-byte records of those candidates only, a batch of 192..256 at a
// time, while it walks the previous batch. A sparse band (few of its tile's
// pairs reach it, and its pixels stop late) then pays one record-gather
// latency per batch of candidates instead of one per 256 pairs of its list.
// Each batch is tested (pixel box, Eq. 4) and compacted exactly as in
// blend_band, in list order, so every pixel's result is bitwise the same.
constexpr int kCandBulk = 4;   // blocks of 64 keys per bulk

template <bool LUT>
VY_DEV void blend_band_keys(Stage& S, uint32_t* __restrict__ cand, int w, int tx, int ty, int band, int half,
                            uint32_t pb, uint32_t pe, const uint32_t* __restrict__ tkey,
                            const uint32_t* __restrict__ tval, const float4* __restrict__ pg0,
                            const float4* __restrict__ pg1, const float4* __restrict__ pg2,
                            const float* __restrict__ prelax, uint32_t n_g, const RCam& cam,
                            float* __restrict__ img, int walk, const ExpLut& L) {
  const int l = (int)(threadIdx.x & 63);
  const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + band * 4 + (l >> 4);
  const bool inside = px < cam.W && py < cam.H && (half < 0 || (l & 15) >> 3 == half);
  PixAcc A;
  pix_init(A, inside);
  const SplitOut so{};
  const float fxp = px + 0.5f, fyp = py + 0.5f;
  const float xa = tx * kTileSize + 0.5f, ya = ty * kTileSize + band * 4 + 0.5f;
  const float xh = half > 0 ? xa + 8.f : xa, xw = half < 0 ? 15.f : 7.f;
  // the job's pixels in tile-local columns and rows, for the key boxes
  const uint32_t cxl = half > 0 ? 8u : 0u, cxh = half == 0 ? 7u : 15u;
  const uint32_t ryl = (uint32_t)band * 4u, ryh = ryl + 3u;
  // key bulks: a = the one being scanned (block qi next), b = the one after
  uint32_t ka[kCandBulk], va[kCandBulk], kb[kCandBulk], vb[kCandBulk];
  uint32_t bulk = pb;   // first position of bulk a
  int qi = 0;
#pragma unroll
  for (int q = 0; q < kCandBulk; ++q) {
    const uint32_t p0 = pb + q * 64 + l, p1 = p0 + 64 * kCandBulk;
    ka[q] = p0 < pe ? tkey[p0] : 0u;
    va[q] = p0 < pe ? tval[p0] : 0u;
    kb[q] = p1 < pe ? tkey[p1] : 0u;
    vb[q] = p1 < pe ? tval[p1] : 0u;
  }
  // collects the next batch of candidates' cut positions into cand[0, n)
  auto assemble = [&]() -> int {
    int n = 0;
    for (;;) {
      const uint32_t sp = bulk + (uint32_t)qi * 64u;
      if (sp >= pe) break;
      uint32_t k = ka[0], v = va[0];
#pragma unroll
      for (int q = 1; q < kCandBulk; ++q) {
        k = qi == q ? ka[q] : k;
        v = qi == q ? va[q] : v;
      }
      const uint32_t bx = k >> 16;
      const bool c = sp + l < pe && (bx & 15u) <= cxh && ((bx >> 4) & 15u) >= cxl && ((bx >> 8) & 15u) <= ryh &&
                     (bx >> 12) >= ryl;
      const uint64_t bal = __ballot(c);
      const int m = __popcll(bal);
      if (n + m > 256) break;   // this block opens the next batch
      if (c) cand[n + __popcll(bal & lanemask_lt())] = v;
      n += m;
      if (++qi == kCandBulk) {   // bulk a done: b becomes a, the one after b is loaded
        qi = 0;
        bulk += 64u * kCandBulk;
#pragma unroll
        for (int q = 0; q < kCandBulk; ++q) {
          ka[q] = kb[q];
          va[q] = vb[q];
          const uint32_t p = bulk + 64u * kCandBulk + q * 64 + l;
          kb[q] = p < pe ? tkey[p] : 0u;
          vb[q] = p < pe ? tval[p] : 0u;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return n;
  };
  // records of a batch's candidates: lane l holds slots h * 64 + l
  float4 qa[kBandParts], qb[kBandParts], qc[kBandParts];
  float qr[kBandParts];
#pragma unroll
  for (int h = 0; h < kBandParts; ++h) {
    qa[h] = qb[h] = qc[h] = make_float4(0.f, 0.f, 0.f, 0.f);
    qr[h] = 1.f;
  }
  auto gather = [&](int n) {
#pragma unroll
    for (int h = 0; h < kBandParts; ++h) {
      const int j = h * 64 + l;
      if (j < n) {
        uint32_t g = cand[j];
        if (g >= n_g) g = 0;
        qa[h] = pg0[g];
        qb[h] = pg1[g];
        qc[h] = pg2[g];
        qr[h] = prelax[g];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();   // cand is read before the next assembly overwrites it
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  int cnt = assemble();
  gather(cnt);
  while (cnt > 0) {
    if (__ballot(!A.done) == 0ull) break;
    // the batch's exact tests and compaction, in list order
    uint32_t base = 0;
#pragma unroll
    for (int h = 0; h < kBandParts; ++h) {
      const int j = h * 64 + l;
      bool hit = j < cnt && band_hit(qa[h].x, qa[h].y, qc[h].w, xh, ya, xw);
      if (hit && qr[h] < 0.25f)   // Eq. 4 over the job's pixel centres, as in blend_band
        hit = rect_rho_max(qa[h].x, qa[h].y, qa[h].z, qa[h].w, qb[h].x, xh, ya, xh + xw, ya + 3.f) * (1.f - qr[h]) >=
              qb[h].z;
      const uint64_t bal = __ballot(hit);
      if (hit) {
        const uint32_t pos = base + (uint32_t)__popcll(bal & lanemask_lt());
        const uint32_t ex = __float_as_uint(qc[h].w);
        S.list[w][pos] = (depth_bin(qb[h].w) << 8) | (uint32_t)j;
        S.r0[w][pos] = qa[h];
        S.r1[w][pos] = make_float4(qb[h].x, qb[h].y, qb[h].z, (float)(ex >> 16));
        S.r2[w][pos] = make_float4(qc[h].x, qc[h].y, qc[h].z, (float)(ex & 0xFFFFu));
      }
      base += (uint32_t)__popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the next batch's candidates, and their records in flight during the walk
    const int next = assemble();
    gather(next);
    const int m = (int)base;
    for (int jc = 0; jc < m; jc += 64) {
      if (__ballot(!A.done) == 0ull) break;
      walk_chunk<true, false, false, LUT>(S, w, jc, m - jc < 64 ? m - jc : 64, 0u, xa, ya, fxp, fyp, A, so, walk, L);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cnt = next;
  }
  if (inside) pixel_out<false>(A, cam, px, py, pb, pe, img, nullptr, nullptr, nullptr, nullptr);
}

// BATCH: the tiles are the global tiles of a batch of views (ntiles in all);
// each job finds its view (camera, image) from the views' first tiles.
template <bool FILTER, bool SAVE, bool LUT, bool BATCH>
__global__ __launch_bounds__(256) void blend_jobs(const uint2* __restrict__ ranges, const uint32_t* __restrict__ tkey,
                                                  const uint32_t* __restrict__ tval,
                                                  const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                                                  const float4* __restrict__ pg2, const float* __restrict__ prelax,
                                                  RCam cam, int ntiles,
                                                  const uint32_t* __restrict__ tile_flag,
                                                  const uint32_t* __restrict__ tiers,
                                                  const uint32_t* __restrict__ heavy_rec,
                                                  const uint4* __restrict__ jobs, float4* __restrict__ bin_c,
                                                  int32_t* __restrict__ bin_n, uint32_t* ctr, uint32_t n_g,
                                                  uint32_t n_pairs_cap, float* __restrict__ img,
                                                  float* __restrict__ Tout, int32_t* __restrict__ Nout,
                                                  int32_t* __restrict__ Eout, int32_t* __restrict__ Lout, int walk,
                                                  int band_wgs, int half_bands, int lut_m,
                                                  const BView* __restrict__ views, int nv) {
  __shared__ Stage S;
  __shared__ uint32_t s_job;
  __shared__ float s_lut[LUT ? kLutMax + 1 : 1];
  __shared__ uint32_t s_toff[BATCH ? kMaxViews + 1 : 1];
  __shared__ uint32_t s_cand[FILTER && !SAVE ? 4 * 256 : 1];   // band jobs' candidate batches, per wave
  ExpLut L{s_lut, 0.f, 0};
  if (LUT) {
    // table values in double, rounded once to float
    for (int k = threadIdx.x; k <= lut_m; k += blockDim.x) s_lut[k] = (float)exp(-kLutRange * k / lut_m);
    L.scale = (float)(lut_m / kLutRange);
    L.m = lut_m;
  }
  if (BATCH) {
    for (int v = threadIdx.x; v < nv; v += blockDim.x) s_toff[v] = views[v].tile_base;
    if (threadIdx.x == 0) s_toff[nv] = (uint32_t)ntiles;
  }
  if (LUT || BATCH) __syncthreads();
  uint32_t njobs = ctr[C_NJOBS];
  if (njobs > kMaxHeavy * kMaxJobsPerTile) njobs = kMaxHeavy * kMaxJobsPerTile;
  const uint32_t n0 = ctr[C_NTIER], n1 = ctr[C_NTIER + 1], n2 = ctr[C_NTIER + 2];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if ((int)blockIdx.x < band_wgs) {
    // the first band_wgs workgroups: every wave takes (tile, band[, half])
    // jobs of the two heaviest tiers on its own, at the highest issue priority
    const uint32_t shift = half_bands ? 3u : 2u;   // jobs per tile: 8 halves or 4 bands
    const uint32_t nband = (n0 + n1) << shift;
    __builtin_amdgcn_s_setprio(3);
    for (;;) {
      uint32_t jb = 0;
      if (l == 0) jb = fetch_add(ctr + C_BAND_TICKET, 1u);
      jb = (uint32_t)__builtin_amdgcn_readfirstlane(jb);
      if (jb >= nband) break;
      const uint32_t k = jb >> shift;
      const int band = (int)((jb >> (shift - 2u)) & 3u), half = half_bands ? (int)(jb & 1u) : -1;
      const uint32_t tile = k < n0 ? tiers[k] : tiers[(size_t)ntiles + (k - n0)];
      const uint2 rg = ranges[tile];
      uint32_t pb = rg.x, pe = rg.y;
      if (pe > n_pairs_cap) pe = n_pairs_cap;
      if (pb > pe) pb = pe;
      RCam vc = cam;
      float* vimg = img;
      uint32_t lt = tile;
      if (BATCH) {
        const int v = __builtin_amdgcn_readfirstlane(view_of(s_toff, nv, tile));
        vc = views[v].cam;
        vimg = views[v].img;
        lt = tile - s_toff[v];
      }
      if (FILTER && !SAVE)
        blend_band_keys<LUT>(S, s_cand + (FILTER && !SAVE ? w * 256 : 0), w, (int)lt % vc.tiles_x,
                             (int)lt / vc.tiles_x, band, half, pb, pe, tkey, tval, pg0, pg1, pg2, prelax, n_g, vc,
                             vimg, walk, L);
      else
        blend_band<FILTER, SAVE, LUT>(S, w, (int)lt % vc.tiles_x, (int)lt / vc.tiles_x, band, half, pb, pe, tval,
                                      pg0, pg1, pg2, prelax, n_g, vc, vimg, Tout, Nout, Eout, Lout, walk, L);
    }
    __builtin_amdgcn_s_setprio(0);
    return;
  }
  // tile jobs: split jobs, the heavy-first tiers not taken by band jobs, then
  // every other tile in order
  const uint32_t nt0 = band_wgs > 0 ? 0u : n0 + n1;
  const uint32_t nfirst = njobs + nt0 + n2;
  const uint32_t total = nfirst + (uint32_t)ntiles;
  for (;;) {
    if (threadIdx.x == 0) s_job = fetch_add(ctr + C_JOB_TICKET, 1u);
    __syncthreads();
    const uint32_t J = s_job;
    if (J >= total) break;
    const bool split = J < njobs;
    uint32_t tile, pb, pe;
    SplitOut so;
    so.bin_c = bin_c;
    so.bin_n = bin_n;
    so.bkey = nullptr;
    so.slot_base = so.lbin0 = so.lbin1 = 0;
    if (split) {
      const uint4 jb = jobs[J];
      const uint32_t* rec = heavy_rec + (size_t)jb.x * kHeavyRec;
      tile = rec[0];
      so.slot_base = rec[2];
      so.lbin0 = jb.y;
      so.lbin1 = jb.z;
      pb = rec[4 + so.lbin0];
      pe = rec[4 + so.lbin1];
      so.bkey = rec + 4 + kMaxBins + 1 + so.lbin0;
    } else {
      if (J < nfirst) {             // heavy-first tiers
        uint32_t k = J - njobs;
        const uint32_t* tl = tiers;
        if (band_wgs > 0) {
          tl += 2 * (size_t)ntiles;
        } else if (k >= n0) {
          k -= n0;
          tl += ntiles;
          if (k >= n1) {
            k -= n1;
            tl += ntiles;
          }
        }
        tile = tl[k];
      } else {
        tile = J - nfirst;
        if (tile_flag[tile] != 0) {   // split, or already blended as a heavy-first tile
          __syncthreads();
          continue;
        }
      }
      const uint2 rg = ranges[tile];
      pb = rg.x;
      pe = rg.y;
    }
    if (pe > n_pairs_cap) pe = n_pairs_cap;
    if (pb > pe) pb = pe;
    RCam vc = cam;
    float* vimg = img;
    uint32_t lt = tile;
    if (BATCH) {
      const int v = __builtin_amdgcn_readfirstlane(view_of(s_toff, nv, tile));
      vc = views[v].cam;
      vimg = views[v].img;
      lt = tile - s_toff[v];
    }
    const int tx = (int)lt % vc.tiles_x, ty = (int)lt / vc.tiles_x;
    const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + w * 4 + (l >> 4);
    const bool inside = px < vc.W && py < vc.H;
    so.pix = (w * 4 + (l >> 4)) * kTileSize + (l & 15);   // row-major in the tile
    PixAcc A;
    pix_init(A, inside);
    A.lb = so.lbin0;
    const float fxp = px + 0.5f, fyp = py + 0.5f;
    // tiles on the critical path (split jobs and the heavy-first tiers) get the
    // highest wave issue priority while they are blended
    const bool urgent = J < nfirst;
    if (urgent) __builtin_amdgcn_s_setprio(3);
    if (split) {
      blend_range<FILTER, true, false, LUT>(S, pb, pe, tval, pg0, pg1, pg2, n_g, tx, ty, fxp, fyp, A, so, 1, L);
      // the current bin, then bins without Gaussians for this band up to the job's end
      if (A.cur_key != 0xFFFFFFFFu && A.lb < so.lbin1) {
        put_bin(so, A.lb, make_float4(A.Cb0, A.Cb1, A.Cb2, A.Tb), A.nb);
        ++A.lb;
      }
      for (; A.lb < so.lbin1; ++A.lb) put_bin(so, A.lb, make_float4(0.f, 0.f, 0.f, 1.f), 0);
    } else {
      blend_range<FILTER, false, SAVE, LUT>(S, pb, pe, tval, pg0, pg1, pg2, n_g, tx, ty, fxp, fyp, A, so, walk, L);
      if (inside) pixel_out<SAVE>(A, vc, px, py, pb, pe, vimg, Tout, Nout, Eout, Lout);
    }
    if (urgent) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
  }
}

// Composite of split tiles, step 1 (one workgroup per heavy tile, one thread
// per pixel): combine the per-bin results in depth order up to the bin in
// which the pixel's blending stops. Pixels that never stop are written here;
// the others record (stop bin, C, T, n) for step 2, and every bin in which
// some pixel stops becomes a redo unit.
struct PixState {
  float4 c;       // C.rgb and T before the stop bin
  int32_t n;
  uint32_t stop;  // stop bin, 0xFFFFFFFF when blending never stops
};

template <bool SAVE>
__global__ __launch_bounds__(256) void composite_scan(RCam cam, const uint32_t* __restrict__ tile_flag,
                                                      const uint32_t* __restrict__ heavy_rec,
                                                      const float4* __restrict__ bin_c,
                                                      const int32_t* __restrict__ bin_n, uint32_t* ctr,
                                                      PixState* __restrict__ pstate, uint2* __restrict__ redo,
                                                      float* __restrict__ img, float* __restrict__ Tout,
                                                      int32_t* __restrict__ Nout, int32_t* __restrict__ Eout) {
  __shared__ uint32_t s_stop[kMaxBins / 32];
  uint32_t nh = ctr[C_NHEAVY];
  if (nh > kMaxHeavy) nh = kMaxHeavy;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const uint32_t* rec = heavy_rec + (size_t)h * kHeavyRec;
    const uint32_t tile = rec[0];
    if (tile_flag[tile] != h + 2) continue;   // blended in one piece (uniform)
    const uint32_t nbins = rec[1], slot_base = rec[2];
    if (threadIdx.x < kMaxBins / 32) s_stop[threadIdx.x] = 0;
    __syncthreads();
    const int tx = (int)tile % cam.tiles_x, ty = (int)tile / cam.tiles_x;
    const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + w * 4 + (l >> 4);
    const bool inside = px < cam.W && py < cam.H;
    const int pix = (w * 4 + (l >> 4)) * kTileSize + (l & 15);
    float Tt = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int32_t nt = 0;
    uint32_t stop = 0xFFFFFFFFu;
    if (inside) {
      for (uint32_t b = 0; b < nbins; ++b) {
        const size_t o = ((size_t)(slot_base + b)) * 256 + pix;
        const float4 r = bin_c[o];
        const int32_t nn = bin_n[o];
        if (Tt * r.w < kTMin) {
          stop = b;
          break;
        }
        C0 = fmaf(Tt, r.x, C0);
        C1 = fmaf(Tt, r.y, C1);
        C2 = fmaf(Tt, r.z, C2);
        Tt = Tt * r.w;
        nt += nn;
      }
      if (stop == 0xFFFFFFFFu) {
        const size_t hw = (size_t)cam.W * cam.H, o = (size_t)py * cam.W + px;
        img[o] = fmaf(Tt, cam.bg[0], C0);
        img[hw + o] = fmaf(Tt, cam.bg[1], C1);
        img[2 * hw + o] = fmaf(Tt, cam.bg[2], C2);
        if (SAVE) {
          Tout[o] = Tt;
          Nout[o] = nt;
          Eout[o] = -1;
        }
      } else {
        atomicOr(&s_stop[stop >> 5], 1u << (stop & 31));
      }
    }
    PixState ps;
    ps.c = make_float4(C0, C1, C2, Tt);
    ps.n = nt;
    ps.stop = stop;
    pstate[(size_t)h * 256 + pix] = ps;
    __syncthreads();
    if (threadIdx.x < kMaxBins / 32) {
      uint32_t m = s_stop[threadIdx.x];
      while (m) {
        const uint32_t bb = threadIdx.x * 32 + (uint32_t)(__ffs(m) - 1);
        m &= m - 1;
        const uint32_t u = fetch_add(ctr + C_NREDO, 1u);
        if (u < kMaxBinSlots) redo[u] = make_uint2(h, bb);
      }
    }
    __syncthreads();
  }
}

// Composite step 2, one workgroup per redo unit (heavy tile h, bin b): the
// pixels whose blending stops in bin b re-blend it from LDS-staged batches
// with their true transmittance and are written.
template <bool FILTER, bool SAVE>
__global__ __launch_bounds__(256) void composite_redo(const uint32_t* __restrict__ tval,
                                                      const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                                                      const float4* __restrict__ pg2, RCam cam,
                                                      const uint32_t* __restrict__ heavy_rec,
                                                      const PixState* __restrict__ pstate,
                                                      const uint2* __restrict__ redo, const uint32_t* ctr,
                                                      uint32_t n_g, uint32_t n_pairs_cap, float* __restrict__ img,
                                                      float* __restrict__ Tout, int32_t* __restrict__ Nout,
                                                      int32_t* __restrict__ Eout, int walk) {
  __shared__ Stage S;
  uint32_t nu = ctr[C_NREDO];
  if (nu > kMaxBinSlots) nu = kMaxBinSlots;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  SplitOut so{};
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    const uint2 unit = redo[u];
    const uint32_t h = unit.x, b = unit.y;
    const uint32_t* rec = heavy_rec + (size_t)h * kHeavyRec;
    const uint32_t tile = rec[0];
    const int tx = (int)tile % cam.tiles_x, ty = (int)tile / cam.tiles_x;
    const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + w * 4 + (l >> 4);
    const int pix = (w * 4 + (l >> 4)) * kTileSize + (l & 15);
    const PixState ps = pstate[(size_t)h * 256 + pix];
    const bool mine = ps.stop == b && px < cam.W && py < cam.H;
    PixAcc A;
    A.Tt = ps.c.w;
    A.C0 = ps.c.x;
    A.C1 = ps.c.y;
    A.C2 = ps.c.z;
    A.nt = ps.n;
    A.Tb = 1.f;
    A.Cb0 = A.Cb1 = A.Cb2 = 0.f;
    A.nb = 0;
    A.stop_pos = 0xFFFFFFFFu;
    A.done = !mine;
    A.cur_key = rec[4 + kMaxBins + 1 + b];   // every pair of the bin has this key: no bin change
    A.lb = 0;
    uint32_t pb = rec[4 + b], pe = rec[4 + b + 1];
    if (pe > n_pairs_cap) pe = n_pairs_cap;
    if (pb > pe) pb = pe;
    blend_range<FILTER, false, false, false>(S, pb, pe, tval, pg0, pg1, pg2, n_g, tx, ty, px + 0.5f, py + 0.5f, A,
                                             so, walk, ExpLut{});
    if (mine) {
      A.C0 = fmaf(A.Tt, A.Cb0, A.C0);
      A.C1 = fmaf(A.Tt, A.Cb1, A.C1);
      A.C2 = fmaf(A.Tt, A.Cb2, A.C2);
      A.Tt = A.Tt * A.Tb;
      A.nt += A.nb;
      const size_t hw = (size_t)cam.W * cam.H, o = (size_t)py * cam.W + px;
      img[o] = fmaf(A.Tt, cam.bg[0], A.C0);
      img[hw + o] = fmaf(A.Tt, cam.bg[1], A.C1);
      img[2 * hw + o] = fmaf(A.Tt, cam.bg[2], A.C2);
      if (SAVE) {
        Tout[o] = A.Tt;
        Nout[o] = A.nt;
        Eout[o] = -1;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Backward pass. The image is C = sum_i c_i alpha_i T_i + T_final bg with
// T_i = prod_{j<i} (1 - alpha_j) over the Gaussians a pixel blended (Eq. 3).
// Walking them back to front from the last one, T_i = T_{i+1} / (1 - alpha_i)
// and with S_i = sum_{j>i} c_j alpha_j T_j + T_final bg (what lies behind i):
//   dC/dc_i = alpha_i T_i,   dC/dalpha_i = c_i T_i - S_i / (1 - alpha_i).
// alpha = min(0.99, theta e^rho) and rho = min(0, A dx^2 + B dx dy + C dy^2)
// (dx = mean - pixel centre) carry it to theta, the 2D mean and (A, B, C);
// the clamps pass no gradient. Per Gaussian, the nine sums are reduced over
// each wave and added into per-cut-position accumulators.
struct GradAcc {
  float* v[9];   // d/d mean2d.x, mean2d.y, A, B, C, theta, r, g, b
};

__global__ __launch_bounds__(256) void bwd_zero(GradAcc acc, const int32_t* n_cut_ptr, uint32_t gcap) {
  uint32_t n = (uint32_t)*n_cut_ptr;
  if (n > gcap) n = gcap;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
#pragma unroll
    for (int k = 0; k < 9; ++k) acc.v[k][i] = 0.f;
}

// Sum of x over the 64 lanes of a fully active wave, complete in lane 63:
// butterflies within quads, mirrors within rows of 16, then the row
// broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3
// (DPP, no LDS traffic). A lane outside the enabled rows adds 0.
template <int CTRL, int ROWS>
VY_DEV float dpp_plus(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}
VY_DEV float wave_sum_to_last(float x) {
  x = dpp_plus<0xB1, 0xF>(x);    // quad_perm [1, 0, 3, 2]
  x = dpp_plus<0x4E, 0xF>(x);    // quad_perm [2, 3, 0, 1]
  x = dpp_plus<0x141, 0xF>(x);   // row_half_mirror
  x = dpp_plus<0x140, 0xF>(x);   // row_mirror: every lane holds its row's sum
  x = dpp_plus<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_plus<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

// The forward's decision at one entry for the pixel centre (fxp, fyp) and,
// when the entry was blended there, its nine gradient terms (d/d mean2d.x,
// mean2d.y, A, B, C, theta, r, g, b); walking back to front, T becomes the
// transmittance in front of the entry and S the colour behind it.
VY_DEV bool entry_grad(const float4 p0, const float4 p1, const float4 p2, float fxp, float fyp, bool in_range,
                       float d0, float d1, float d2, float& T, float& S0, float& S1, float& S2, float v[9]) {
  const float dx = p0.x - fxp, dy = p0.y - fyp;
  const float raw = fmaf(dx, fmaf(p0.z, dx, p0.w * dy), (p1.x * dy) * dy);
  const float power = fminf(raw, 0.f);
  const uint32_t ext = __float_as_uint(p2.w);
  bool on = in_range && fabsf(dx) <= (float)(ext & 0xFFFFu) && fabsf(dy) <= (float)(ext >> 16);
  const float e = __expf(power);
  const float araw = p1.y * e;
  const float alpha = fminf(kAlphaMax, araw);
  on = on && alpha >= kAlphaMin;   // the forward's decision, recomputed the same way
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = 0.f;
  if (on) {
    const float om = 1.f - alpha;
    T = T / om;                                          // transmittance in front of this Gaussian
    const float wgt = alpha * T;
    v[6] = wgt * d0;
    v[7] = wgt * d1;
    v[8] = wgt * d2;
    const float io = 1.f / om;
    const float dla = (p2.x * T - S0 * io) * d0 + (p2.y * T - S1 * io) * d1 + (p2.z * T - S2 * io) * d2;
    S0 = fmaf(p2.x, wgt, S0);
    S1 = fmaf(p2.y, wgt, S1);
    S2 = fmaf(p2.z, wgt, S2);
    if (araw < kAlphaMax) {
      v[5] = dla * e;                                    // d alpha / d theta = e^rho
      if (raw < 0.f) {
        const float gr = dla * alpha;                    // d alpha / d rho = alpha
        v[0] = gr * fmaf(2.f * p0.z, dx, p0.w * dy);
        v[1] = gr * fmaf(p0.w, dx, 2.f * p1.x * dy);
        v[2] = gr * dx * dx;
        v[3] = gr * dx * dy;
        v[4] = gr * dy * dy;
      }
    }
  }
  return on;
}

// One wave per (tile, band of 16x4 pixels) job: the wave walks its tile's
// list back to front in chunks of 64, from the band's furthest last
// contributor, over the entries whose pixel box may reach the band. Every lane
// repeats the forward's decision for its pixel. A chunk is walked in one of
// two ways, with the same per-pixel arithmetic in the same order:
//   - together (most entries cover most pixels of the band): entry by entry,
//     the nine sums are reduced across the wave when several lanes contribute
//     (else each contributing lane adds its own) and added atomically at the
//     entry's cut position;
//   - per pixel (far, small Gaussians): each lane walks only the entries whose
//     pixel box holds its pixel centre, back to front, adding its terms into
//     per-entry LDS sums, which are then added at the entries' cut positions.
__global__ __launch_bounds__(256) void blend_backward(const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ tval,
                                                      const float4* __restrict__ pg0, const float4* __restrict__ pg1,
                                                      const float4* __restrict__ pg2, RCam cam, int ntiles,
                                                      const float* __restrict__ dimg, const float* __restrict__ Tfin,
                                                      const int32_t* __restrict__ last, uint32_t n_g,
                                                      uint32_t n_pairs_cap, GradAcc acc) {
  __shared__ float4 s_r[4][3][64];
  __shared__ uint32_t s_g[4][64];
  __shared__ float s_acc[4][9][64];   // per-entry sums of the per-pixel walk
  const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
  const size_t hw = (size_t)cam.W * cam.H;
  const int njobs = 4 * ntiles;
  for (int job = blockIdx.x * 4 + w; job < njobs; job += gridDim.x * 4) {
    const int tile = job >> 2, band = job & 3;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * kTileSize + (l & 15), py = ty * kTileSize + band * 4 + (l >> 4);
    const bool inside = px < cam.W && py < cam.H;
    const size_t o = (size_t)py * cam.W + px;
    const uint2 rg = ranges[tile];
    uint32_t pb = rg.x, pe = rg.y;
    if (pe > n_pairs_cap) pe = n_pairs_cap;
    if (pb > pe) pb = pe;
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, T = 1.f;
    int lst = -1;
    if (inside) {
      d0 = dimg[o];
      d1 = dimg[hw + o];
      d2 = dimg[2 * hw + o];
      T = Tfin[o];
      lst = last[o];
    }
    float S0 = T * cam.bg[0], S1 = T * cam.bg[1], S2 = T * cam.bg[2];
    int wl = lst;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) wl = max(wl, __shfl_xor(wl, s, 64));
    const int pend = wl + 1;   // wave-uniform: nothing past the band's last contributor
    const float fxp = px + 0.5f, fyp = py + 0.5f;
    const float xa = tx * kTileSize + 0.5f, ya = ty * kTileSize + band * 4 + 0.5f;
    for (int bend = pend; bend > (int)pb; bend -= 64) {
      const int b0 = bend - 64 > (int)pb ? bend - 64 : (int)pb;
      const int cnt = bend - b0;
      bool hit = false;
      float bx = 0.f, by = 0.f, brx = -1.f, bry = -1.f;   // this lane's entry's pixel box (empty if none)
      if (l < cnt) {
        uint32_t g = tval[b0 + l];
        if (g >= n_g) g = 0;
        const float4 a = pg0[g], b = pg1[g], c = pg2[g];
        hit = band_hit(a.x, a.y, c.w, xa, ya);
        s_r[w][0][l] = a;
        s_r[w][1][l] = b;
        s_r[w][2][l] = c;
        s_g[w][l] = g;
        if (hit) {
          const uint32_t ext = __float_as_uint(c.w);
          bx = a.x;
          by = a.y;
          brx = (float)(ext & 0xFFFFu);
          bry = (float)(ext >> 16);
        }
      }
      uint64_t mask = ballot(hit);
      // per lane: the chunk's entries whose box holds the lane's pixel centre
      // (the pixel rule, with the same float expressions), up to its last contributor
      const int cc = l & 15, cr = l >> 4;
      uint64_t mc = 0ull, mr = 0ull;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const uint64_t bb = ballot(fabsf(bx - (xa + (float)i)) <= brx);
        mc = cc == i ? bb : mc;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t bb = ballot(fabsf(by - (ya + (float)i)) <= bry);
        mr = cr == i ? bb : mr;
      }
      uint64_t mk = mc & mr;
      const int lim = lst - b0;   // entries j <= lim may have been blended at this pixel
      mk = lim < 0 ? 0ull : (lim >= 63 ? mk : mk & ((2ull << lim) - 1ull));
      const int pc = __popcll(mk);
      int mx = 0;
#pragma unroll
      for (int bt = 6; bt >= 0; --bt)
        if (ballot(pc >= (mx | (1 << bt))) != 0ull) mx |= 1 << bt;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // per pixel when the busiest pixel needs under 70 % of the band's entries
      // (measured: 35 % 2.9 ms, 50 % 2.0, 70 % 1.86, 85 % 1.92, always 2.1 per 1080p frame)
      if (mx * 10 < __popcll(mask) * 7) {
        // per pixel: each lane over its own entries, back to front
#pragma unroll
        for (int k = 0; k < 9; ++k) s_acc[w][k][l] = 0.f;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        while (ballot(mk != 0ull) != 0ull) {
          if (mk != 0ull) {
            const int j = 63 - __builtin_clzll(mk);
            mk &= ~(1ull << j);
            float v[9];
            if (entry_grad(s_r[w][0][j], s_r[w][1][j], s_r[w][2][j], fxp, fyp, true, d0, d1, d2, T, S0, S1, S2,
                           v)) {
#pragma unroll
              for (int k = 0; k < 9; ++k)
                if (v[k] != 0.f) atomicAdd(&s_acc[w][k][j], v[k]);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (l < cnt) {
          const uint32_t g = s_g[w][l];
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            const float x = s_acc[w][k][l];
            if (x != 0.f) atomicAdd(acc.v[k] + g, x);
          }
        }
      } else {
        // together: entry by entry, back to front
        while (mask != 0ull) {
          const int j = 63 - __builtin_clzll(mask);
          mask &= ~(1ull << j);
          float v[9];
          const bool on = entry_grad(s_r[w][0][j], s_r[w][1][j], s_r[w][2][j], fxp, fyp, b0 + j <= lst, d0, d1,
                                     d2, T, S0, S1, S2, v);
          const uint64_t onm = ballot(on);
          if (onm == 0ull) continue;
          const uint32_t g = s_g[w][j];
          if (__popcll(onm) <= 2) {
            if (on) {
#pragma unroll
              for (int k = 0; k < 9; ++k)
                if (v[k] != 0.f) atomicAdd(acc.v[k] + g, v[k]);
            }
          } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) v[k] = wave_sum_to_last(v[k]);
            if (l == 63) {
#pragma unroll
              for (int k = 0; k < 9; ++k)
                if (v[k] != 0.f) atomicAdd(acc.v[k] + g, v[k]);
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// Gradients of the SH colour's basis (the forward's polynomial forms) at the
// unit direction (x, y, z): rows are d Y_k / d(x, y, z).
VY_DEV void sh_basis_grad(float x, float y, float z, float Y[16], float G[16][3]) {
  const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f, C2a = 1.0925484305920792f;
  const float C20 = 0.31539156525252005f, C22 = 0.5462742152960396f, C33 = 0.5900435899266435f;
  const float C32 = 2.890611442640554f, C31 = 0.4570457994644658f, C30 = 0.3731763325901154f;
  const float C32p = 1.445305721320277f;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = C0;            G[0][0] = 0.f;                G[0][1] = 0.f;                 G[0][2] = 0.f;
  Y[1] = C1 * y;        G[1][0] = 0.f;                G[1][1] = C1;                  G[1][2] = 0.f;
  Y[2] = C1 * z;        G[2][0] = 0.f;                G[2][1] = 0.f;                 G[2][2] = C1;
  Y[3] = C1 * x;        G[3][0] = C1;                 G[3][1] = 0.f;                 G[3][2] = 0.f;
  Y[4] = C2a * x * y;   G[4][0] = C2a * y;            G[4][1] = C2a * x;             G[4][2] = 0.f;
  Y[5] = C2a * y * z;   G[5][0] = 0.f;                G[5][1] = C2a * z;             G[5][2] = C2a * y;
  Y[6] = C20 * (3.f * zz - 1.f);
  G[6][0] = 0.f;        G[6][1] = 0.f;                G[6][2] = 6.f * C20 * z;
  Y[7] = C2a * x * z;   G[7][0] = C2a * z;            G[7][1] = 0.f;                 G[7][2] = C2a * x;
  Y[8] = C22 * (xx - yy);
  G[8][0] = 2.f * C22 * x;  G[8][1] = -2.f * C22 * y;  G[8][2] = 0.f;
  Y[9] = C33 * y * (3.f * xx - yy);
  G[9][0] = 6.f * C33 * x * y;  G[9][1] = 3.f * C33 * (xx - yy);  G[9][2] = 0.f;
  Y[10] = C32 * x * y * z;
  G[10][0] = C32 * y * z;  G[10][1] = C32 * x * z;  G[10][2] = C32 * x * y;
  Y[11] = C31 * y * (5.f * zz - 1.f);
  G[11][0] = 0.f;  G[11][1] = C31 * (5.f * zz - 1.f);  G[11][2] = 10.f * C31 * y * z;
  Y[12] = C30 * z * (5.f * zz - 3.f);
  G[12][0] = 0.f;  G[12][1] = 0.f;  G[12][2] = C30 * (15.f * zz - 3.f);
  Y[13] = C31 * x * (5.f * zz - 1.f);
  G[13][0] = C31 * (5.f * zz - 1.f);  G[13][1] = 0.f;  G[13][2] = 10.f * C31 * x * z;
  Y[14] = C32p * z * (xx - yy);
  G[14][0] = 2.f * C32p * x * z;  G[14][1] = -2.f * C32p * y * z;  G[14][2] = C32p * (xx - yy);
  Y[15] = C33 * x * (xx - 3.f * yy);
  G[15][0] = 3.f * C33 * (xx - yy);  G[15][1] = -6.f * C33 * x * y;  G[15][2] = 0.f;
}

struct NodeGrads {
  float* mean;           // [n][3]
  float* log_scale;      // [n][3]
  float* quat;           // [n][4]
  float* logit;          // [n]
  float* sh;             // [n][48]
  float* mean2d;         // [n][2]
  const float* quat_raw; // [n][4] or null
};

// Per cut Gaussian: the projection (Section 3.1 "Culling & Projection", as in
// `project`) differentiated from the accumulated 2D-mean, conic, opacity and
// colour gradients down to the node's parameters.
__global__ __launch_bounds__(256) void project_backward(const int32_t* __restrict__ cut, const int32_t* n_cut_ptr,
                                                        const float4* __restrict__ gauss,
                                                        const float* __restrict__ sh, RCam cam, GradAcc acc,
                                                        NodeGrads out, int64_t n_nodes, uint32_t gcap) {
  uint32_t n = (uint32_t)*n_cut_ptr;
  if (n > gcap) n = gcap;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const int32_t node = cut[i];
    if (node < 0 || node >= n_nodes) continue;
    float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, glogit = 0.f;
    float gsh[48];
#pragma unroll
    for (int k = 0; k < 48; ++k) gsh[k] = 0.f;
    const float g_mx = acc.v[0][i], g_my = acc.v[1][i];
    const float4 g0 = gauss[3 * (int64_t)node], g1 = gauss[3 * (int64_t)node + 1], g2 = gauss[3 * (int64_t)node + 2];
    const float dxw = g0.x - cam.px, dyw = g0.y - cam.py, dzw = g0.z - cam.pz;
    const float x = (cam.R[0] * dxw + cam.R[1] * dyw) + cam.R[2] * dzw;
    const float y = (cam.R[3] * dxw + cam.R[4] * dyw) + cam.R[5] * dzw;
    const float z = (cam.R[6] * dxw + cam.R[7] * dyw) + cam.R[8] * dzw;
    if (z > cam.near) {
      const float qw = g2.x, qx = g2.y, qy = g2.z, qz = g2.w;
      const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                           2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                           2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
      const float s[3] = {g1.x, g1.y, g1.z};
      const float iz = 1.f / z;
      const float ur = x * iz, vr = y * iz;
      const float u = fminf(fmaxf(ur, cam.ulo), cam.uhi), v = fminf(fmaxf(vr, cam.vlo), cam.vhi);
      float T0[3], T1[3], M[9], V0[3], V1[3];
      for (int k = 0; k < 3; ++k) {
        T0[k] = (cam.fx * iz) * (cam.R[k] - u * cam.R[6 + k]);
        T1[k] = (cam.fy * iz) * (cam.R[3 + k] - v * cam.R[6 + k]);
      }
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) M[3 * r + j] = Rq[3 * r + j] * s[j];
      for (int j = 0; j < 3; ++j) {
        V0[j] = (T0[0] * M[j] + T0[1] * M[3 + j]) + T0[2] * M[6 + j];
        V1[j] = (T1[0] * M[j] + T1[1] * M[3 + j]) + T1[2] * M[6 + j];
      }
      const float a = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + kLowpass;
      const float b = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2];
      const float c = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + kLowpass;
      const float det = fmaf(a, c, -b * b);
      if (det > 0.f) {
        // conic (ca, cb, cc) = (c, -b, a) / det; rho uses (A, B, C) = (-ca/2, -cb, -cc/2)
        const float dca = -0.5f * acc.v[2][i], dcb = -acc.v[3][i], dcc = -0.5f * acc.v[4][i];
        const float id2 = 1.f / (det * det);
        const float ga = (-c * c * dca + b * c * dcb - b * b * dcc) * id2;
        const float gb = (2.f * b * c * dca - (a * c + b * b) * dcb + 2.f * a * b * dcc) * id2;
        const float gc = (-b * b * dca + a * b * dcb - a * a * dcc) * id2;
        // Sigma2 = V V^T (+ low-pass): a = |V0|^2, b = V0.V1, c = |V1|^2
        float gV0[3], gV1[3];
        for (int j = 0; j < 3; ++j) {
          gV0[j] = 2.f * ga * V0[j] + gb * V1[j];
          gV1[j] = gb * V0[j] + 2.f * gc * V1[j];
        }
        // V = T M
        float gT0[3], gT1[3], gM[9];
        for (int k = 0; k < 3; ++k) {
          gT0[k] = (gV0[0] * M[3 * k] + gV0[1] * M[3 * k + 1]) + gV0[2] * M[3 * k + 2];
          gT1[k] = (gV1[0] * M[3 * k] + gV1[1] * M[3 * k + 1]) + gV1[2] * M[3 * k + 2];
          for (int j = 0; j < 3; ++j) gM[3 * k + j] = T0[k] * gV0[j] + T1[k] * gV1[j];
        }
        // M = Rq diag(s): scales (as log-scales) and the rotation
        float gR[9];
        for (int j = 0; j < 3; ++j) {
          const float gs = (gM[j] * Rq[j] + gM[3 + j] * Rq[3 + j]) + gM[6 + j] * Rq[6 + j];
          gls[j] = gs * s[j];
          for (int r = 0; r < 3; ++r) gR[3 * r + j] = gM[3 * r + j] * s[j];
        }
        gq[0] = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
        gq[1] = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                       qw * gR[7] - 2.f * qx * gR[8]);
        gq[2] = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                       qz * gR[7] - 2.f * qy * gR[8]);
        gq[3] = 2.f * (-2.f * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.f * qz * gR[4] + qy * gR[5] +
                       qx * gR[6] + qy * gR[7]);
        // T rows: fx/z (R0 - u R2), fy/z (R1 - v R2); mean2d = (fx x/z + cx, fy y/z + cy)
        float g_iz = g_mx * cam.fx * x + g_my * cam.fy * y, g_u = 0.f, g_v = 0.f;
        for (int k = 0; k < 3; ++k) {
          g_iz += gT0[k] * cam.fx * (cam.R[k] - u * cam.R[6 + k]) + gT1[k] * cam.fy * (cam.R[3 + k] - v * cam.R[6 + k]);
          g_u -= gT0[k] * cam.fx * iz * cam.R[6 + k];
          g_v -= gT1[k] * cam.fy * iz * cam.R[6 + k];
        }
        const bool fu = ur > cam.ulo && ur < cam.uhi, fv = vr > cam.vlo && vr < cam.vhi;   // clamps pass nothing
        float gx = g_mx * cam.fx * iz, gy = g_my * cam.fy * iz;
        if (fu) {
          gx += g_u * iz;
          g_iz += g_u * x;
        }
        if (fv) {
          gy += g_v * iz;
          g_iz += g_v * y;
        }
        const float gz = -g_iz * iz * iz;
        // x_cam = R (mean - pos)
        for (int k = 0; k < 3; ++k) gm[k] = (cam.R[k] * gx + cam.R[3 + k] * gy) + cam.R[6 + k] * gz;
        // opacity: theta = sigmoid(logit)
        const float th = g1.w;
        glogit = acc.v[5][i] * th * (1.f - th);
        // colour: clamp(sum_k Y_k(d) sh_k + 0.5, 0, 1), d = (mean - camera centre) / |.|
        const float dn = 1.f / sqrtf((dxw * dxw + dyw * dyw) + dzw * dzw);
        const float ux = dxw * dn, uy = dyw * dn, uz = dzw * dn;
        float Y[16], G[16][3];
        sh_basis_grad(ux, uy, uz, Y, G);
        const float* cf = sh + 48 * (int64_t)node;
        float raw[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < 16; ++k)
          for (int ch = 0; ch < 3; ++ch) raw[ch] = fmaf(Y[k], cf[3 * k + ch], raw[ch]);
        float gcol[3];
        for (int ch = 0; ch < 3; ++ch) {
          const float cr = raw[ch] + 0.5f;
          gcol[ch] = (cr > 0.f && cr < 1.f) ? acc.v[6 + ch][i] : 0.f;
        }
        float gd[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < 16; ++k) {
          float w = 0.f;
          for (int ch = 0; ch < 3; ++ch) {
            gsh[3 * k + ch] = Y[k] * gcol[ch];
            w = fmaf(cf[3 * k + ch], gcol[ch], w);
          }
          for (int e = 0; e < 3; ++e) gd[e] = fmaf(w, G[k][e], gd[e]);
        }
        const float rad = (ux * gd[0] + uy * gd[1]) + uz * gd[2];
        gm[0] += (gd[0] - ux * rad) * dn;
        gm[1] += (gd[1] - uy * rad) * dn;
        gm[2] += (gd[2] - uz * rad) * dn;
      }
    }
    // the unit quaternion came from the caller's q / |q|
    if (out.quat_raw) {
      const float* qr = out.quat_raw + 4 * (int64_t)node;
      const float nq = sqrtf((qr[0] * qr[0] + qr[1] * qr[1]) + (qr[2] * qr[2] + qr[3] * qr[3]));
      const float in = 1.f / nq;
      const float qh[4] = {qr[0] * in, qr[1] * in, qr[2] * in, qr[3] * in};
      const float dot = (qh[0] * gq[0] + qh[1] * gq[1]) + (qh[2] * gq[2] + qh[3] * gq[3]);
      for (int k = 0; k < 4; ++k) gq[k] = (gq[k] - qh[k] * dot) * in;
    }
    if (out.mean)
      for (int k = 0; k < 3; ++k) out.mean[3 * (int64_t)node + k] = gm[k];
    if (out.log_scale)
      for (int k = 0; k < 3; ++k) out.log_scale[3 * (int64_t)node + k] = gls[k];
    if (out.quat)
      for (int k = 0; k < 4; ++k) out.quat[4 * (int64_t)node + k] = gq[k];
    if (out.logit) out.logit[node] = glogit;
    if (out.sh)
      for (int k = 0; k < 48; ++k) out.sh[48 * (int64_t)node + k] = gsh[k];
    if (out.mean2d) {
      out.mean2d[2 * (int64_t)node] = g_mx;
      out.mean2d[2 * (int64_t)node + 1] = g_my;
    }
  }
}

RCam make_rcam(const vy_camera* c, const vy_render_opts* opt) {
  RCam r;
  for (int i = 0; i < 9; ++i) r.R[i] = c->R[i];
  r.px = c->pos[0];
  r.py = c->pos[1];
  r.pz = c->pos[2];
  r.fx = c->fx;
  r.fy = c->fy;
  r.cx = c->cx;
  r.cy = c->cy;
  r.near = c->znear;
  r.W = c->width;
  r.H = c->height;
  r.ulo = -kClamp * c->cx / c->fx;
  r.uhi = kClamp * ((float)c->width - c->cx) / c->fx;
  r.vlo = -kClamp * c->cy / c->fy;
  r.vhi = kClamp * ((float)c->height - c->cy) / c->fy;
  r.tiles_x = (c->width + kTileSize - 1) / kTileSize;
  r.tiles_y = (c->height + kTileSize - 1) / kTileSize;
  for (int k = 0; k < 3; ++k) r.bg[k] = opt ? opt->bg[k] : 0.f;
  r.ln_amin = logf(kAlphaMin);
  // With the LUT the exponential is read at the nearest table node, up to half
  // an interval (5.55 / 2m) above rho: the check keeps that much more margin so
  // that the filtered image stays identical to the unfiltered one.
  const int m = opt ? opt->lut_entries : 0;
  r.fdelta = kFilterDelta + (m > 0 ? (float)(kLutRange / (2.0 * m)) * 1.001f : 0.f);
  return r;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int imin(int64_t a, int64_t b) { return (int)(a < b ? a : b); }

// ------------------------------------------------------------------------
// Frame summary for the serving runtime: an order-independent 64-bit hash of
// the image's bits, the sum over flat index i of mix64(i << 32 | bits(image[i]))
// modulo 2^64 (mix64 is the finaliser of Steele, Lea and Flood's SplitMix64),
// so that any changed value changes the hash, plus the frame's counts and
// error flags. The record must be zero before the launch (the hash is summed
// with one atomic add per workgroup).
struct FrameStats {
  unsigned long long hash;
  uint32_t n_cut, n_pairs, n_visible, flags, n_frontier, pad;
};
static_assert(sizeof(FrameStats) == 32, "frame record layout");

VY_DEV uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void frame_finish(const uint32_t* __restrict__ img, uint32_t n,
                                                    const int32_t* n_front, const int32_t* n_cut,
                                                    const uint32_t* cut_err, const uint32_t* ctr,
                                                    FrameStats* out) {
  __shared__ unsigned long long s_part[4];
  unsigned long long acc = 0;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
    acc += mix64(((uint64_t)i << 32) | img[i]);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane() == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&out->hash, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
    if (blockIdx.x == 0) {
      out->n_cut = (uint32_t)*n_cut;
      out->n_frontier = (uint32_t)*n_front;
      out->n_pairs = ctr[C_NPAIRS_RAW];
      out->n_visible = ctr[C_NVIS];
      out->flags = (ctr[C_OVERFLOW] ? 1u : 0u) | (ctr[C_GOVER] ? 2u : 0u) | (ctr[C_ERR] ? 4u : 0u) |
                   (*cut_err ? 8u : 0u);
    }
  }
}

}  // namespace

using namespace vy;

extern "C" {

static int64_t status_words_for(int64_t max_g, int64_t max_pairs) {
  const int64_t a = cdiv(max_pairs, vysort::kTile), b = cdiv(max_g, vysort::kTile);
  return (a > b ? a : b) * 256 + 256;
}

size_t vy_render_workspace_bytes(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs) {
  return render_workspace_bytes(max_g, max_w, max_h, max_pairs, true);
}

}  // extern "C"

namespace vy {

size_t render_workspace_bytes(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs, bool split) {
  if (max_g < 1 || max_w < 1 || max_h < 1 || max_pairs < 1) return 0;
  const int64_t tiles = cdiv(max_w, kTileSize) * cdiv(max_h, kTileSize);
  size_t b = 0;
  b += (size_t)max_g * (16 * 4 + 4 * 7);   // pg0..2, prec, relax, big, offsets, dkey x2, dval x2
  b += (size_t)max_pairs * 4 * 4;                          // tkey x2, tval x2
  b += (size_t)tiles * 8;
  b += 64 * 4 + 6 * 256 * 4;
  b += (size_t)status_words_for(max_g, max_pairs) * 8;
  b += (size_t)max_w * max_h * 16;                         // saved T, n_contrib, n_eval, last contributor
  b += (size_t)tiles * 16;                                 // tile flags, tiers
  if (split) {                                             // tiles split by depth bins
    b += kMaxHeavy * 4 + (size_t)kMaxHeavy * kHeavyRec * 4 + (size_t)kMaxHeavy * kMaxJobsPerTile * 16;
    b += (size_t)kMaxBinSlots * (256 * 20 + 4 + 8);        // per-bin results, slot owners, redo units
    b += (size_t)kMaxHeavy * 256 * sizeof(PixState);
  }
  b += 32 * 256;
  return b;
}

}  // namespace vy

extern "C" {

int vy_render_ctx_create(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs, void* ws, size_t bytes,
                         vy_render_ctx** out) {
  return render_ctx_create_on(max_g, max_w, max_h, max_pairs, true, ws, bytes, nullptr, true, out);
}

}  // extern "C"

namespace vy {

__global__ void zero_words(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Clears n 32-bit words with a kernel (a memset node recorded into a captured
// graph is avoided: callers of the no-allocation entry point may capture it).
static int zero_on(void* p, int64_t words, hipStream_t st) {
  zero_words<<<imin(cdiv(words, 256), 1024), 256, 0, st>>>((uint32_t*)p, words);
  VY_LAUNCHED();
  return VY_OK;
}

// Lays the context's buffers out in `ws` and enqueues the clearing of what must
// start at zero (look-back words, counters). No host or device allocation.
static int render_ctx_carve(RenderCtx* c, int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs,
                            bool split, void* ws, size_t bytes, hipStream_t st) {
  if (!ws || max_g < 1 || max_w < 1 || max_h < 1 || max_pairs < 1 || max_pairs > 0x7FFFFFFF ||
      max_g > 0x7FFFFFFF || max_w > 32768 || max_h > 32768)
    return fail(VY_ERR_ARG, "vy_render_ctx_create: bad argument");
  if (cdiv(max_w, kTileSize) * cdiv(max_h, kTileSize) > 65536)
    return fail(VY_ERR_ARG, "vy_render_ctx_create: more than 65536 tiles (16-bit tile keys)");
  const size_t need = render_workspace_bytes(max_g, max_w, max_h, max_pairs, split);
  if (bytes < need) return fail(VY_ERR_ARG, "vy_render_ctx_create: workspace %zu < %zu bytes", bytes, need);
  *c = RenderCtx();
  Carver cv(ws, bytes);
  c->magic = kCtxMagic;
  c->max_g = max_g;
  c->max_pairs = max_pairs;
  c->max_w = max_w;
  c->max_h = max_h;
  c->max_tiles = cdiv(max_w, kTileSize) * cdiv(max_h, kTileSize);
  c->pg0 = cv.take<float4>(max_g);
  c->pg1 = cv.take<float4>(max_g);
  c->pg2 = cv.take<float4>(max_g);
  c->prec = cv.take<uint4>(max_g);
  c->prelax = cv.take<float>(max_g);
  c->big = cv.take<uint32_t>(max_g);
  c->offsets = cv.take<uint32_t>(max_g);
  c->dkey[0] = cv.take<uint32_t>(max_g);
  c->dkey[1] = cv.take<uint32_t>(max_g);
  c->dval[0] = cv.take<uint32_t>(max_g);
  c->dval[1] = cv.take<uint32_t>(max_g);
  c->tkey[0] = cv.take<uint32_t>(max_pairs);
  c->tkey[1] = cv.take<uint32_t>(max_pairs);
  c->tval[0] = cv.take<uint32_t>(max_pairs);
  c->tval[1] = cv.take<uint32_t>(max_pairs);
  c->ranges = cv.take<uint2>(c->max_tiles);
  c->ctr = cv.take<uint32_t>(64);
  c->hist = cv.take<uint32_t>(6 * 256);
  c->status_words = status_words_for(max_g, max_pairs);
  c->status = cv.take<uint64_t>(c->status_words);
  c->T_final = cv.take<float>((size_t)max_w * max_h);
  c->tile_flag = cv.take<uint32_t>(c->max_tiles);
  c->tiers = cv.take<uint32_t>(3 * c->max_tiles);
  c->split = split;
  if (split) {
    c->heavy_list = cv.take<uint32_t>(kMaxHeavy);
    c->heavy_rec = cv.take<uint32_t>((size_t)kMaxHeavy * kHeavyRec);
    c->jobs = cv.take<uint4>((size_t)kMaxHeavy * kMaxJobsPerTile);
    c->slot_owner = cv.take<uint32_t>(kMaxBinSlots);
    c->pstate_raw = cv.take<PixState>((size_t)kMaxHeavy * 256);
    c->redo = cv.take<uint2>(kMaxBinSlots);
    c->bin_c = cv.take<float4>((size_t)kMaxBinSlots * 256);
    c->bin_n = cv.take<int32_t>((size_t)kMaxBinSlots * 256);
  }
  c->n_contrib = cv.take<int32_t>((size_t)max_w * max_h);
  c->n_eval = cv.take<int32_t>((size_t)max_w * max_h);
  c->last_contrib = cv.take<int32_t>((size_t)max_w * max_h);
  if (!cv.ok()) {
    c->magic = 0;
    return fail(VY_ERR_ARG, "vy_render_ctx_create: workspace layout overflow");
  }
  if (int rc = zero_on(c->status, 2 * c->status_words, st)) return rc;
  if (int rc = zero_on(c->ctr, 64, st)) return rc;
  c->epoch = 0;
  return VY_OK;
}

int render_ctx_create_on(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs, bool split, void* ws,
                         size_t bytes, hipStream_t st, bool sync, vy_render_ctx** out) {
  if (!out) return fail(VY_ERR_ARG, "vy_render_ctx_create: bad argument");
  RenderCtx* c = (RenderCtx*)calloc(1, sizeof(RenderCtx));
  if (!c) return fail(VY_ERR_ARG, "vy_render_ctx_create: out of host memory");
  if (int rc = render_ctx_carve(c, max_g, max_w, max_h, max_pairs, split, ws, bytes, st)) {
    free(c);
    return rc;
  }
  if (sync) {
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      free(c);
      return fail(VY_ERR_HIP, "vy_render_ctx_create: %s", hipGetErrorString(e));
    }
  }
  *out = (vy_render_ctx*)c;
  return VY_OK;
}

}  // namespace vy

// ------------------------------------------- rendering without allocation ----
// The scratch of vy_render_noalloc: one context's buffers in a static device
// array (each GPU holds its own copy from the first call until the process
// ends), laid out once per device at a fixed capacity. Host code reaches the
// array only through the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) unsigned char scratch[VY_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoallocDevices = 64;
struct NoallocState {
  bool ready = false;
  void* ptr = nullptr;   // this device's address of `scratch`
  RenderCtx ctx;
};
NoallocState g_noalloc[kNoallocDevices];
std::mutex g_noalloc_mu;

__global__ void noalloc_counts(const uint32_t* __restrict__ ctr, uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = ctr[C_NPAIRS_RAW];
    out[1] = ctr[C_NVIS];
    out[2] = ctr[C_GOVER];
    out[3] = ctr[C_ERR];
  }
}
}  // namespace

extern "C" {

int vy_render_ctx_free(vy_render_ctx* ctx) {
  RenderCtx* c = (RenderCtx*)ctx;
  if (!c) return VY_OK;
  if (c->magic != kCtxMagic) return fail(VY_ERR_ARG, "vy_render_ctx_free: not a render context");
  c->magic = 0;
  free(c);
  return VY_OK;
}

static int epoch_for(RenderCtx* c, hipStream_t st, uint32_t* ep) {
  *ep = next_epoch(c->epoch);
  if (*ep == 1) return zero_on(c->status, 2 * c->status_words, st);
  return VY_OK;
}

static int render_impl(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
                       float* image, vy_render_ctx* ctx, void* stream);

int vy_render(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
              float* image, vy_render_ctx* ctx, void* stream) {
  return render_impl(scene, cut, cam, opts, image, ctx, stream);
}

int vy_render_noalloc(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
                      float* image, uint32_t* counts, void* stream) {
  if (!cam || !image) return fail(VY_ERR_ARG, "vy_render_noalloc: bad argument");
  if (cam->width < 1 || cam->height < 1 || cam->width > VY_NOALLOC_MAX_WIDTH || cam->height > VY_NOALLOC_MAX_HEIGHT)
    return fail(VY_ERR_ARG, "vy_render_noalloc: image %dx%d exceeds the static scratch's %dx%d", cam->width,
                cam->height, VY_NOALLOC_MAX_WIDTH, VY_NOALLOC_MAX_HEIGHT);
  if (opts && (opts->save_state || opts->split_min_pairs > 0))
    return fail(VY_ERR_ARG, "vy_render_noalloc: save_state and split tiles need a render context (vy_render)");
  int dev = 0;
  VY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocDevices) return fail(VY_ERR_ARG, "vy_render_noalloc: device %d not supported", dev);
  hipStream_t st = (hipStream_t)stream;
  NoallocState& g = g_noalloc[dev];
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g.ready) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(VY_ERR_HIP, "vy_render_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      if (int rc = render_ctx_carve(&g.ctx, VY_NOALLOC_MAX_GAUSSIANS, VY_NOALLOC_MAX_WIDTH, VY_NOALLOC_MAX_HEIGHT,
                                    VY_NOALLOC_MAX_PAIRS, false, ptr, VY_NOALLOC_SCRATCH_BYTES, st))
        return rc;
      g.ptr = ptr;
      g.ready = true;
    }
  }
  if (int rc = render_impl(scene, cut, cam, opts, image, (vy_render_ctx*)&g.ctx, stream)) return rc;
  if (counts) {
    noalloc_counts<<<1, 64, 0, st>>>(g.ctx.ctr, counts);
    VY_LAUNCHED();
  }
  return VY_OK;
}

// ------------------------------------------------------ batched frames ----

size_t vy_batch_workspace_bytes(int32_t max_views, int64_t max_g, int64_t max_tiles, int64_t max_pairs) {
  if (max_views < 1 || max_views > VY_BATCH_MAX_VIEWS || max_g < 1 || max_tiles < 1 ||
      max_tiles > VY_BATCH_MAX_TILES || max_pairs < 1)
    return 0;
  size_t b = 0;
  b += (size_t)max_g * (16 * 4 + 4 * 7);
  b += (size_t)max_pairs * 4 * 4;
  b += (size_t)max_tiles * (8 + 16);
  b += 64 * 4 + 6 * 256 * 4;
  b += (size_t)status_words_for(max_g, max_pairs) * 8;
  b += (size_t)kMaxViews * (sizeof(BView) + 4) + 4;
  b += 32 * 256;
  return b;
}

namespace {
constexpr int kBatchRing = 4;
constexpr uint32_t kBatchMagic = 0x56594254u;
struct BatchCtx {
  uint32_t magic;
  RenderCtx c;              // the shared buffers (no per-pixel state, no split tiles)
  int max_views;
  BView* d_views;           // device descriptor of the current batch
  uint32_t* d_goff;         // device [max_views + 1]
  BView* h_views[kBatchRing];   // pinned host copies, one per call in a ring
  hipEvent_t copied[kBatchRing];
  int slot;
};
}  // namespace

int vy_batch_ctx_create(int32_t max_views, int64_t max_g, int64_t max_tiles, int64_t max_pairs, void* ws,
                        size_t bytes, vy_batch_ctx** out) {
  const size_t need = vy_batch_workspace_bytes(max_views, max_g, max_tiles, max_pairs);
  if (!ws || !out || need == 0 || max_g > 0x7FFFFFFF || max_pairs > 0x7FFFFFFF)
    return fail(VY_ERR_ARG, "vy_batch_ctx_create: bad argument");
  if (bytes < need) return fail(VY_ERR_ARG, "vy_batch_ctx_create: workspace %zu < %zu bytes", bytes, need);
  BatchCtx* b = new (std::nothrow) BatchCtx();
  if (!b) return fail(VY_ERR_ARG, "vy_batch_ctx_create: out of host memory");
  RenderCtx* c = &b->c;
  Carver cv(ws, bytes);
  c->magic = kCtxMagic;
  c->max_g = max_g;
  c->max_pairs = max_pairs;
  c->max_tiles = max_tiles;
  c->pg0 = cv.take<float4>(max_g);
  c->pg1 = cv.take<float4>(max_g);
  c->pg2 = cv.take<float4>(max_g);
  c->prec = cv.take<uint4>(max_g);
  c->prelax = cv.take<float>(max_g);
  c->big = cv.take<uint32_t>(max_g);
  c->offsets = cv.take<uint32_t>(max_g);
  c->dkey[0] = cv.take<uint32_t>(max_g);
  c->dkey[1] = cv.take<uint32_t>(max_g);
  c->dval[0] = cv.take<uint32_t>(max_g);
  c->dval[1] = cv.take<uint32_t>(max_g);
  c->tkey[0] = cv.take<uint32_t>(max_pairs);
  c->tkey[1] = cv.take<uint32_t>(max_pairs);
  c->tval[0] = cv.take<uint32_t>(max_pairs);
  c->tval[1] = cv.take<uint32_t>(max_pairs);
  c->ranges = cv.take<uint2>(max_tiles);
  c->ctr = cv.take<uint32_t>(64);
  c->hist = cv.take<uint32_t>(6 * 256);
  c->status_words = status_words_for(max_g, max_pairs);
  c->status = cv.take<uint64_t>(c->status_words);
  c->tile_flag = cv.take<uint32_t>(max_tiles);
  c->tiers = cv.take<uint32_t>(3 * max_tiles);
  b->d_views = cv.take<BView>(kMaxViews);
  b->d_goff = cv.take<uint32_t>(kMaxViews + 1);
  b->max_views = max_views;
  int rc = VY_OK;
  if (!cv.ok()) rc = fail(VY_ERR_ARG, "vy_batch_ctx_create: workspace layout overflow");
  for (int k = 0; k < kBatchRing && rc == VY_OK; ++k) {
    if (hipHostMalloc((void**)&b->h_views[k], sizeof(BView) * kMaxViews, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming) != hipSuccess)
      rc = fail(VY_ERR_HIP, "vy_batch_ctx_create: pinned descriptor or event");
  }
  if (rc == VY_OK) rc = zero_on(c->status, 2 * c->status_words, nullptr);
  if (rc == VY_OK) rc = zero_on(c->ctr, 64, nullptr);
  if (rc == VY_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(VY_ERR_HIP, "vy_batch_ctx_create: sync");
  if (rc != VY_OK) {
    for (int k = 0; k < kBatchRing; ++k) {
      if (b->h_views[k]) (void)hipHostFree(b->h_views[k]);
      if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
    }
    delete b;
    return rc;
  }
  b->magic = kBatchMagic;
  *out = (vy_batch_ctx*)b;
  return VY_OK;
}

int vy_batch_ctx_free(vy_batch_ctx* ctx) {
  BatchCtx* b = (BatchCtx*)ctx;
  if (!b) return VY_OK;
  if (b->magic != kBatchMagic) return fail(VY_ERR_ARG, "vy_batch_ctx_free: not a batch context");
  b->magic = 0;
  for (int k = 0; k < kBatchRing; ++k) {
    (void)hipEventSynchronize(b->copied[k]);
    (void)hipHostFree(b->h_views[k]);
    (void)hipEventDestroy(b->copied[k]);
  }
  delete b;
  return VY_OK;
}

int vy_render_batch(const vy_view* views, int32_t n, const vy_render_opts* opts, vy_batch_ctx* ctx, void* stream) {
  BatchCtx* b = (BatchCtx*)ctx;
  if (!b || b->magic != kBatchMagic || !views || n < 1 || n > b->max_views)
    return fail(VY_ERR_ARG, "vy_render_batch: bad argument (n_views %d)", n);
  if (opts && (opts->save_state || opts->split_min_pairs > 0))
    return fail(VY_ERR_ARG, "vy_render_batch: save_state and split tiles are for single frames (vy_render)");
  const int walk = opts ? opts->walk : 0;
  if (walk < 0 || walk > 2) return fail(VY_ERR_ARG, "vy_render_batch: walk must be 0, 1 or 2");
  const int band_jobs = opts ? opts->band_jobs : 0;
  if (band_jobs < 0 || band_jobs > 2) return fail(VY_ERR_ARG, "vy_render_batch: band_jobs must be 0, 1 or 2");
  // a batch is throughput work: the whole-band layout unless asked otherwise
  const bool half_bands = band_jobs == 1;
  if (opts && (opts->lut_entries < 0 || opts->lut_entries > kLutMax))
    return fail(VY_ERR_ARG, "vy_render_batch: lut_entries must be 0..%d", kLutMax);
  RenderCtx* c = &b->c;
  hipStream_t st = (hipStream_t)stream;
  const int slot = b->slot = (b->slot + 1) % kBatchRing;
  VY_HIP(hipEventSynchronize(b->copied[slot]));   // the copy of this ring slot's last batch has been read
  BView* hv = b->h_views[slot];
  uint32_t tiles = 0;
  for (int v = 0; v < n; ++v) {
    const vy_view& q = views[v];
    const Scene* s = (const Scene*)q.scene;
    const Cut* ct = (const Cut*)q.cut;
    if (!s || s->magic != kSceneMagic || !ct || ct->magic != kCutMagic || !q.image)
      return fail(VY_ERR_ARG, "vy_render_batch: view %d: bad scene, cut or image", v);
    if (ct->scene != s) return fail(VY_ERR_ARG, "vy_render_batch: view %d: cut belongs to another scene", v);
    if (ct->cur < 0) return fail(VY_ERR_STATE, "vy_render_batch: view %d: cut has not been computed", v);
    if (q.cam.width < 1 || q.cam.height < 1 || q.cam.width > 32768 || q.cam.height > 32768 || !(q.cam.fx > 0.f) ||
        !(q.cam.fy > 0.f) || !(q.cam.znear > 0.f))
      return fail(VY_ERR_ARG, "vy_render_batch: view %d: invalid camera", v);
    BView& o = hv[v];
    o.cam = make_rcam(&q.cam, opts);
    o.gauss = s->gauss;
    o.sh = s->sh;
    o.cut = cut_ids_dev(ct);
    o.n_cut = cut_count_dev(ct);
    o.n_nodes = s->n;
    o.img = q.image;
    o.tile_base = tiles;
    o.pad = 0;
    const uint64_t t = (uint64_t)tiles + (uint64_t)o.cam.tiles_x * (uint64_t)o.cam.tiles_y;
    if (t > (uint64_t)c->max_tiles)
      return fail(VY_ERR_ARG, "vy_render_batch: the views' %llu tiles exceed the context's %lld",
                  (unsigned long long)t, (long long)c->max_tiles);
    tiles = (uint32_t)t;
  }
  VY_HIP(hipMemcpyAsync(b->d_views, hv, sizeof(BView) * n, hipMemcpyHostToDevice, st));
  VY_HIP(hipEventRecord(b->copied[slot], st));
  const bool filter = opts && opts->alpha_filter;
  const int lut_m = opts ? opts->lut_entries : 0;
  const int ntiles = (int)tiles;
  const uint32_t gcap = (uint32_t)c->max_g, pcap = (uint32_t)c->max_pairs;
  const ViewsRef vr{b->d_views, b->d_goff, n};
  int tile_bits = 1;
  while ((1 << tile_bits) < ntiles) ++tile_bits;
  const int bits0 = (tile_bits + 1) / 2, bits1 = tile_bits - bits0;
  {
    ProfScope ps(VY_STAGE_RENDER_SETUP, st);
    batch_setup<<<16, 256, 0, st>>>(b->d_views, n, b->d_goff, gcap, c->ctr, c->hist, c->ranges, ntiles);
    VY_LAUNCHED();
  }
  {
    ProfScope ps(VY_STAGE_PROJECT, st);
    const int blocks = imin(cdiv(c->max_g, 256), 512);
    if (filter)
      project_batch<true><<<blocks, 256, 0, st>>>(b->d_views, b->d_goff, n, c->pg0, c->pg1, c->pg2, c->prec,
                                                  c->prelax, c->dkey[0], c->ctr, c->hist, c->big);
    else
      project_batch<false><<<blocks, 256, 0, st>>>(b->d_views, b->d_goff, n, c->pg0, c->pg1, c->pg2, c->prec,
                                                   c->prelax, c->dkey[0], c->ctr, c->hist, c->big);
    VY_LAUNCHED();
    if (filter) {
      big_count<true><<<512, 256, 0, st>>>(c->big, c->ctr, c->pg0, c->pg1, c->prec, c->prelax, 0, 0, gcap, vr);
      VY_LAUNCHED();
    }
  }
  {
    const int blocks = imin(cdiv(c->max_g, vysort::kTile), 256);
    const uint32_t* n_all = b->d_goff + n;   // the batch's Gaussians
    for (int p = 0; p < 4; ++p) {
      ProfScope ps(VY_STAGE_DEPTH_SORT, st);
      uint32_t ep;
      if (int rcode = epoch_for(c, st, &ep)) return rcode;
      const uint32_t* kin = c->dkey[p & 1];
      const uint32_t* vin = p == 0 ? nullptr : c->dval[p & 1];
      vysort::onesweep_pass<<<blocks, vysort::kThreads, 0, st>>>(
          kin, vin, c->dkey[(p + 1) & 1], c->dval[(p + 1) & 1], n_all, gcap, 8 * p, 255u, 8, c->hist + 256 * p,
          c->status, ep, c->ctr + C_TICKET0 + p, c->ctr + C_ERR);
      VY_LAUNCHED();
    }
  }
  {
    ProfScope ps(VY_STAGE_EMIT, st);
    uint32_t ep;
    if (int rcode = epoch_for(c, st, &ep)) return rcode;
    const int blocks = imin(cdiv(c->max_g, kScanTile), 512);
    pair_emit<true><<<blocks, 256, 0, st>>>(c->dval[0], c->prec, c->offsets, c->ctr, c->status, ep, 0, bits0,
                                            c->tkey[0], c->tval[0], c->hist, pcap, gcap, vr);
    VY_LAUNCHED();
    if (filter)
      emit_big<true, true><<<512, 256, 0, st>>>(c->big, c->offsets, c->prec, c->pg0, c->pg1, c->prelax, 0, 0, 0,
                                                bits0, c->tkey[0], c->tval[0], c->ctr, c->hist, pcap, gcap, vr);
    else
      emit_big<false, true><<<512, 256, 0, st>>>(c->big, c->offsets, c->prec, c->pg0, c->pg1, c->prelax, 0, 0, 0,
                                                 bits0, c->tkey[0], c->tval[0], c->ctr, c->hist, pcap, gcap, vr);
    VY_LAUNCHED();
  }
  {
    const int blocks = imin(cdiv(c->max_pairs, vysort::kTile), 256);
    const uint32_t* np = c->ctr + C_NPAIRS;
    for (int p = 0; p < 2; ++p) {
      ProfScope ps(VY_STAGE_TILE_SORT, st);
      uint32_t ep;
      if (int rcode = epoch_for(c, st, &ep)) return rcode;
      const int shift = p == 0 ? 0 : bits0;
      const int nb = p == 0 ? bits0 : bits1;
      const uint32_t mask = nb > 0 ? ((1u << nb) - 1u) : 0u;
      vysort::onesweep_pass<<<blocks, vysort::kThreads, 0, st>>>(
          c->tkey[p & 1], c->tval[p & 1], c->tkey[(p + 1) & 1], c->tval[(p + 1) & 1], np, pcap, shift, mask, nb,
          c->hist + 256 * (4 + p), c->status, ep, c->ctr + C_TICKET0 + 4 + p, c->ctr + C_ERR);
      VY_LAUNCHED();
    }
  }
  {
    ProfScope ps(VY_STAGE_RANGES, st);
    const int blocks = imin(cdiv(c->max_pairs, 1024), 4096);
    tile_ranges<<<blocks, 256, 0, st>>>(c->tkey[0], c->ctr, c->ranges, (uint32_t)ntiles);
    VY_LAUNCHED();
  }
  const int band_wgs = walk != 0 ? 0 : half_bands ? kBandWGsLatency : kBandWGsThroughput;
  {
    ProfScope ps(VY_STAGE_BLEND_PLAN, st);
    plan_tiles<<<imin(cdiv(ntiles, 256), 64), 256, 0, st>>>(c->ranges, ntiles, c->tile_flag, nullptr, c->tiers,
                                                            c->ctr, 0xFFFFFFFFu);
    VY_LAUNCHED();
  }
  {
    ProfScope ps(VY_STAGE_BLEND, st);
    const RCam none{};
#define VY_BLEND_BATCH(F, LT)                                                                                    \
  blend_jobs<F, false, LT, true><<<band_wgs + 2048, 256, 0, st>>>(                                             \
      c->ranges, c->tkey[0], c->tval[0], c->pg0, c->pg1, c->pg2, c->prelax, none, ntiles, c->tile_flag,         \
      c->tiers, nullptr, nullptr, nullptr, nullptr, c->ctr, gcap, pcap, nullptr, nullptr, nullptr, nullptr,      \
      nullptr, walk, band_wgs, half_bands, lut_m, b->d_views, n)
    if (filter) {
      if (lut_m > 0) VY_BLEND_BATCH(true, true); else VY_BLEND_BATCH(true, false);
    } else {
      if (lut_m > 0) VY_BLEND_BATCH(false, true); else VY_BLEND_BATCH(false, false);
    }
#undef VY_BLEND_BATCH
    VY_LAUNCHED();
  }
  return VY_OK;
}

int vy_batch_status(vy_batch_ctx* ctx, int64_t* n_pairs, int64_t* n_visible, void* stream) {
  BatchCtx* b = (BatchCtx*)ctx;
  if (!b || b->magic != kBatchMagic) return fail(VY_ERR_ARG, "vy_batch_status: bad argument");
  return vy_render_status((vy_render_ctx*)&b->c, n_pairs, n_visible, stream);
}

static int render_impl(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
                       float* image, vy_render_ctx* ctx, void* stream) {
  const Scene* s = (const Scene*)scene;
  const Cut* ct = (const Cut*)cut;
  RenderCtx* c = (RenderCtx*)ctx;
  if (!s || s->magic != kSceneMagic || !ct || ct->magic != kCutMagic || !c || c->magic != kCtxMagic || !cam ||
      !image)
    return fail(VY_ERR_ARG, "vy_render: bad argument");
  if (ct->scene != s) return fail(VY_ERR_ARG, "vy_render: cut belongs to another scene");
  if (ct->cur < 0) return fail(VY_ERR_STATE, "vy_render: cut has not been computed");
  if (cam->width < 1 || cam->height < 1 || cam->width > c->max_w || cam->height > c->max_h)
    return fail(VY_ERR_ARG, "vy_render: image %dx%d exceeds the context (%dx%d)", cam->width, cam->height,
                c->max_w, c->max_h);
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !(cam->znear > 0.f))
    return fail(VY_ERR_ARG, "vy_render: invalid camera intrinsics");
  const bool filter = opts && opts->alpha_filter;
  const bool save = opts && opts->save_state;
  const int walk = opts ? opts->walk : 0;
  if (walk < 0 || walk > 2) return fail(VY_ERR_ARG, "vy_render: walk must be 0, 1 or 2");
  const int band_jobs = opts ? opts->band_jobs : 0;
  if (band_jobs < 0 || band_jobs > 2) return fail(VY_ERR_ARG, "vy_render: band_jobs must be 0, 1 or 2");
  const bool half_bands = band_jobs != 2;   // one frame: the latency layout unless asked otherwise
  if (opts && (opts->lut_entries < 0 || opts->lut_entries > kLutMax))
    return fail(VY_ERR_ARG, "vy_render: lut_entries must be 0..%d", kLutMax);
  if (opts && opts->lut_entries > 0 && opts->split_min_pairs > 0)
    return fail(VY_ERR_ARG, "vy_render: split tiles are blended with the exact exponential only");
  hipStream_t st = (hipStream_t)stream;
  const RCam rc = make_rcam(cam, opts);
  const int ntiles = rc.tiles_x * rc.tiles_y;
  const int32_t* cut_ids = cut_ids_dev(ct);
  const uint32_t* n_cut = (const uint32_t*)cut_count_dev(ct);
  const uint32_t gcap = (uint32_t)c->max_g, pcap = (uint32_t)c->max_pairs;
  int tile_bits = 1;
  while ((1 << tile_bits) < ntiles) ++tile_bits;
  const int bits0 = (tile_bits + 1) / 2, bits1 = tile_bits - bits0;
  {
    ProfScope ps(VY_STAGE_RENDER_SETUP, st);
    render_setup<<<16, 256, 0, st>>>(c->ctr, c->hist, c->ranges, ntiles);
    VY_LAUNCHED();
  }
  {
    ProfScope ps(VY_STAGE_PROJECT, st);
    // 512 workgroups: more pay in per-block histogram flushes (256..10240 measured)
    const int blocks = imin(cdiv(c->max_g, 256), 512);
    if (filter)
      project<true><<<blocks, 256, 0, st>>>(cut_ids, (const int32_t*)n_cut, s->gauss, s->sh, rc, c->pg0, c->pg1,
                                            c->pg2, c->prec, c->prelax, c->dkey[0], c->ctr,
                                            c->hist, s->n, c->big, gcap);
    else
      project<false><<<blocks, 256, 0, st>>>(cut_ids, (const int32_t*)n_cut, s->gauss, s->sh, rc, c->pg0, c->pg1,
                                             c->pg2, c->prec, c->prelax, c->dkey[0], c->ctr,
                                             c->hist, s->n, c->big, gcap);
    VY_LAUNCHED();
    if (filter) {
      big_count<false><<<512, 256, 0, st>>>(c->big, c->ctr, c->pg0, c->pg1, c->prec, c->prelax, rc.W, rc.H, gcap,
                                            ViewsRef{});
      VY_LAUNCHED();
    }
  }
  {
    // depth sort of all cut entries (culled ones carry key 0xFFFFFFFF and sort last)
    const int blocks = imin(cdiv(c->max_g, vysort::kTile), 256);
    for (int p = 0; p < 4; ++p) {
      ProfScope ps(VY_STAGE_DEPTH_SORT, st);
      uint32_t ep;
      if (int rcode = epoch_for(c, st, &ep)) return rcode;
      const uint32_t* kin = c->dkey[p & 1];
      const uint32_t* vin = p == 0 ? nullptr : c->dval[p & 1];
      vysort::onesweep_pass<<<blocks, vysort::kThreads, 0, st>>>(
          kin, vin, c->dkey[(p + 1) & 1], c->dval[(p + 1) & 1], n_cut, gcap, 8 * p, 255u, 8, c->hist + 256 * p,
          c->status, ep, c->ctr + C_TICKET0 + p, c->ctr + C_ERR);
      VY_LAUNCHED();
    }
  }
  // sorted order now in dkey[0] / dval[0]; the first C_NVIS entries are the visible Gaussians
  {
    // pair scan + emission in depth order, then the big Gaussians' pairs
    ProfScope ps(VY_STAGE_EMIT, st);
    uint32_t ep;
    if (int rcode = epoch_for(c, st, &ep)) return rcode;
    const int blocks = imin(cdiv(c->max_g, kScanTile), 512);
    pair_emit<false><<<blocks, 256, 0, st>>>(c->dval[0], c->prec, c->offsets, c->ctr, c->status, ep, rc.tiles_x,
                                             bits0, c->tkey[0], c->tval[0], c->hist, pcap, gcap, ViewsRef{});
    VY_LAUNCHED();
    if (filter)
      emit_big<true, false><<<512, 256, 0, st>>>(c->big, c->offsets, c->prec, c->pg0, c->pg1, c->prelax, rc.W, rc.H,
                                                 rc.tiles_x, bits0, c->tkey[0], c->tval[0], c->ctr, c->hist, pcap,
                                                 gcap, ViewsRef{});
    else
      emit_big<false, false><<<512, 256, 0, st>>>(c->big, c->offsets, c->prec, c->pg0, c->pg1, c->prelax, rc.W,
                                                  rc.H, rc.tiles_x, bits0, c->tkey[0], c->tval[0], c->ctr, c->hist,
                                                  pcap, gcap, ViewsRef{});
    VY_LAUNCHED();
  }
  {
    const int blocks = imin(cdiv(c->max_pairs, vysort::kTile), 256);
    const uint32_t* np = c->ctr + C_NPAIRS;
    for (int p = 0; p < 2; ++p) {
      ProfScope ps(VY_STAGE_TILE_SORT, st);
      uint32_t ep;
      if (int rcode = epoch_for(c, st, &ep)) return rcode;
      const int shift = p == 0 ? 0 : bits0;
      const int nb = p == 0 ? bits0 : bits1;
      const uint32_t mask = nb > 0 ? ((1u << nb) - 1u) : 0u;
      vysort::onesweep_pass<<<blocks, vysort::kThreads, 0, st>>>(
          c->tkey[p & 1], c->tval[p & 1], c->tkey[(p + 1) & 1], c->tval[(p + 1) & 1], np, pcap, shift, mask, nb,
          c->hist + 256 * (4 + p), c->status, ep, c->ctr + C_TICKET0 + 4 + p, c->ctr + C_ERR);
      VY_LAUNCHED();
    }
  }
  {
    ProfScope ps(VY_STAGE_RANGES, st);
    const int blocks = imin(cdiv(c->max_pairs, 1024), 4096);
    tile_ranges<<<blocks, 256, 0, st>>>(c->tkey[0], c->ctr, c->ranges, (uint32_t)ntiles);
    VY_LAUNCHED();
  }
  // splitting tiles by depth bins gives up early termination; it is off unless asked for
  // automatic walk: the two heaviest tiers are blended band by band by waves of their own
  const int band_wgs = walk != 0 ? 0 : half_bands ? kBandWGsLatency : kBandWGsThroughput;
  const bool split_on = opts && opts->split_min_pairs > 0;
  if (split_on && !c->split) return fail(VY_ERR_ARG, "vy_render: this context has no room for split tiles");
  const int lut_m = opts ? opts->lut_entries : 0;
  // what the backward pass will find saved
  c->saved = save && !split_on && lut_m == 0;
  c->saved_scene = s;
  c->saved_cut = ct;
  c->saved_version = ct->version;
  c->saved_params = s->params_version;
  c->saved_cam = *cam;
  for (int k = 0; k < 3; ++k) c->saved_bg[k] = opts ? opts->bg[k] : 0.f;
  const uint32_t split_min = split_on ? (uint32_t)opts->split_min_pairs : 0xFFFFFFFFu;
  {
    ProfScope ps(VY_STAGE_BLEND_PLAN, st);
    plan_tiles<<<imin(cdiv(ntiles, 256), 64), 256, 0, st>>>(c->ranges, ntiles, c->tile_flag, c->heavy_list,
                                                            c->tiers, c->ctr, split_min);
    VY_LAUNCHED();
    if (split_on) {
      plan_heavy<<<256, 256, 0, st>>>(c->ranges, c->tval[0], c->pg1, c->heavy_list, c->tile_flag, c->heavy_rec,
                                      c->jobs, c->slot_owner, c->ctr, gcap, split_min);
      VY_LAUNCHED();
    }
  }
  {
    ProfScope ps(VY_STAGE_BLEND, st);
#define VY_BLEND_JOBS(F, S, LT)                                                                                 \
  blend_jobs<F, S, LT, false><<<band_wgs + 2048, 256, 0, st>>>(                                                 \
      c->ranges, c->tkey[0], c->tval[0], c->pg0, c->pg1, c->pg2, c->prelax, rc, ntiles, c->tile_flag, c->tiers,  \
      c->heavy_rec, c->jobs, c->bin_c, c->bin_n, c->ctr, gcap, pcap, image, c->T_final, c->n_contrib,            \
      c->n_eval, c->last_contrib, walk, band_wgs, half_bands, lut_m, nullptr, 0)
#define VY_BLEND(F, S)                                                                                          \
  do {                                                                                                          \
    if (lut_m > 0) VY_BLEND_JOBS(F, S, true); else VY_BLEND_JOBS(F, S, false);                                  \
    if (split_on) {                                                                                             \
      composite_scan<S><<<256, 256, 0, st>>>(rc, c->tile_flag, c->heavy_rec, c->bin_c, c->bin_n, c->ctr,           \
                                             reinterpret_cast<PixState*>(c->pstate_raw), c->redo, image,         \
                                             c->T_final, c->n_contrib, c->n_eval);                              \
      composite_redo<F, S><<<2048, 256, 0, st>>>(c->tval[0], c->pg0, c->pg1, c->pg2, rc, c->heavy_rec,             \
                                                 reinterpret_cast<const PixState*>(c->pstate_raw), c->redo, c->ctr, \
                                                 gcap, pcap, image, c->T_final, c->n_contrib, c->n_eval, walk); \
    }                                                                                                           \
  } while (0)
    if (filter) {
      if (save) VY_BLEND(true, true); else VY_BLEND(true, false);
    } else {
      if (save) VY_BLEND(false, true); else VY_BLEND(false, false);
    }
#undef VY_BLEND
#undef VY_BLEND_JOBS
    VY_LAUNCHED();
  }
  return VY_OK;
}

int vy_render_backward(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const float* dL_dimage,
                       const vy_grads* grads, vy_render_ctx* ctx, void* stream) {
  const Scene* s = (const Scene*)scene;
  const Cut* ct = (const Cut*)cut;
  RenderCtx* c = (RenderCtx*)ctx;
  if (!s || s->magic != kSceneMagic || !ct || ct->magic != kCutMagic || !c || c->magic != kCtxMagic || !cam ||
      !dL_dimage || !grads)
    return fail(VY_ERR_ARG, "vy_render_backward: bad argument");
  if (!c->saved)
    return fail(VY_ERR_STATE, "vy_render_backward: the last vy_render on this context did not save its state "
                              "(save_state = 1, no split tiles, exact exponential)");
  if (c->saved_scene != s || c->saved_cut != ct || c->saved_version != ct->version ||
      memcmp(&c->saved_cam, cam, sizeof(vy_camera)) != 0)
    return fail(VY_ERR_STATE, "vy_render_backward: the saved frame is of another scene, cut or camera");
  if (c->saved_params != s->params_version)
    return fail(VY_ERR_STATE, "vy_render_backward: the scene's Gaussians were updated after the saved frame");
  hipStream_t st = (hipStream_t)stream;
  const RCam rc = make_rcam(cam, nullptr);
  RCam rcb = rc;
  for (int k = 0; k < 3; ++k) rcb.bg[k] = c->saved_bg[k];
  const int ntiles = rc.tiles_x * rc.tiles_y;
  const uint32_t gcap = (uint32_t)c->max_g, pcap = (uint32_t)c->max_pairs;
  const int32_t* cut_ids = cut_ids_dev(ct);
  const int32_t* n_cut = cut_count_dev(ct);
  // per-cut-position accumulators in buffers the forward no longer needs
  // (depth-sort keys and values, Gaussian offsets, big list, rounding
  // allowances, binning records)
  float* pr = reinterpret_cast<float*>(c->prec);
  GradAcc acc{{reinterpret_cast<float*>(c->dkey[0]), reinterpret_cast<float*>(c->dkey[1]),
               reinterpret_cast<float*>(c->dval[0]), reinterpret_cast<float*>(c->dval[1]),
               reinterpret_cast<float*>(c->offsets), reinterpret_cast<float*>(c->big), c->prelax, pr,
               pr + c->max_g}};
  const int gblocks = imin(cdiv(c->max_g, 256), 2048);
  {
    ProfScope ps(VY_STAGE_BWD_BLEND, st);
    bwd_zero<<<gblocks, 256, 0, st>>>(acc, n_cut, gcap);
    VY_LAUNCHED();
    blend_backward<<<imin(ntiles, 4096), 256, 0, st>>>(c->ranges, c->tval[0], c->pg0, c->pg1, c->pg2, rcb, ntiles,
                                                       dL_dimage, c->T_final, c->last_contrib, gcap, pcap, acc);
    VY_LAUNCHED();
  }
  {
    ProfScope ps(VY_STAGE_BWD_PROJECT, st);
    NodeGrads out{grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->sh, grads->mean2d,
                  grads->quat_raw};
    project_backward<<<gblocks, 256, 0, st>>>(cut_ids, n_cut, s->gauss, s->sh, rc, acc, out, s->n, gcap);
    VY_LAUNCHED();
  }
  return VY_OK;
}

int vy_render_status(vy_render_ctx* ctx, int64_t* n_pairs, int64_t* n_visible, void* stream) {
  RenderCtx* c = (RenderCtx*)ctx;
  if (!c || c->magic != kCtxMagic) return fail(VY_ERR_ARG, "vy_render_status: bad argument");
  uint32_t h[C_COUNT];
  hipStream_t st = (hipStream_t)stream;
  VY_HIP(hipMemcpyAsync(h, c->ctr, sizeof(h), hipMemcpyDeviceToHost, st));
  VY_HIP(hipStreamSynchronize(st));
  if (n_visible) *n_visible = h[C_NVIS];
  if (h[C_GOVER]) {
    if (n_pairs) *n_pairs = h[C_NPAIRS];
    return fail(VY_ERR_CAPACITY, "vy_render: cut of %u Gaussians exceeds max_gaussians %lld", h[C_GOVER],
                (long long)c->max_g);
  }
  if (h[C_OVERFLOW]) {
    if (n_pairs) *n_pairs = h[C_NPAIRS_RAW];
    return fail(VY_ERR_CAPACITY, "vy_render: %u pairs exceed max_pairs %lld", h[C_NPAIRS_RAW],
                (long long)c->max_pairs);
  }
  if (n_pairs) *n_pairs = h[C_NPAIRS];
  if (h[C_ERR]) return fail(VY_ERR_DEVICE, "vy_render: device-side bound hit (%u)", h[C_ERR]);
  return VY_OK;
}

int vy_render_saved(const vy_render_ctx* ctx, const float** T_final, const int32_t** n_contrib,
                    const int32_t** n_eval, const int32_t** last_contrib, const float** mean2d) {
  const RenderCtx* c = (const RenderCtx*)ctx;
  if (!c || c->magic != kCtxMagic) return fail(VY_ERR_ARG, "vy_render_saved: bad argument");
  if (T_final) *T_final = c->T_final;
  if (n_contrib) *n_contrib = c->n_contrib;
  if (n_eval) *n_eval = c->n_eval;
  if (last_contrib) *last_contrib = c->last_contrib;
  if (mean2d) *mean2d = (const float*)c->pg0;
  return VY_OK;
}

int vy_render_pairs(const vy_render_ctx* ctx, const uint32_t** tile_keys, const uint32_t** cut_pos,
                    const uint32_t** ranges) {
  const RenderCtx* c = (const RenderCtx*)ctx;
  if (!c || c->magic != kCtxMagic) return fail(VY_ERR_ARG, "vy_render_pairs: bad argument");
  if (tile_keys) *tile_keys = c->tkey[0];
  if (cut_pos) *cut_pos = c->tval[0];
  if (ranges) *ranges = reinterpret_cast<const uint32_t*>(c->ranges);
  return VY_OK;
}

int vy_render_projected(const vy_render_ctx* ctx, const float** rec0, const float** rec1, const float** rec2,
                        const uint32_t** bin_rec) {
  const RenderCtx* c = (const RenderCtx*)ctx;
  if (!c || c->magic != kCtxMagic) return fail(VY_ERR_ARG, "vy_render_projected: bad argument");
  if (rec0) *rec0 = reinterpret_cast<const float*>(c->pg0);
  if (rec1) *rec1 = reinterpret_cast<const float*>(c->pg1);
  if (rec2) *rec2 = reinterpret_cast<const float*>(c->pg2);
  if (bin_rec) *bin_rec = reinterpret_cast<const uint32_t*>(c->prec);
  return VY_OK;
}

}  // extern "C"

namespace vy {

int batch_frame_finish(const vy_cut* cut, const vy_batch_ctx* batch, const float* image, int32_t width,
                       int32_t height, void* stats, hipStream_t st) {
  const BatchCtx* b = (const BatchCtx*)batch;
  if (!b || b->magic != kBatchMagic) return fail(VY_ERR_ARG, "frame summary: not a batch context");
  return render_frame_finish(cut, (const vy_render_ctx*)&b->c, image, width, height, stats, st);
}

int render_frame_finish(const vy_cut* cut, const vy_render_ctx* ctx, const float* image, int32_t width,
                        int32_t height, void* stats, hipStream_t st) {
  const Cut* ct = (const Cut*)cut;
  const RenderCtx* c = (const RenderCtx*)ctx;
  if (!ct || ct->magic != kCutMagic || !c || c->magic != kCtxMagic || !image || !stats || width < 1 ||
      height < 1 || width > 32768 || height > 32768)
    return fail(VY_ERR_ARG, "frame summary: bad argument");
  const uint32_t n = 3u * (uint32_t)width * (uint32_t)height;
  frame_finish<<<imin(cdiv(n, 256 * 16), 1024), 256, 0, st>>>((const uint32_t*)image, n,
                                                             cut_frontier_count_dev(ct), cut_count_dev(ct),
                                                             cut_err_dev(ct), c->ctr, (FrameStats*)stats);
  VY_LAUNCHED();
  return VY_OK;
}

}  // namespace vy
