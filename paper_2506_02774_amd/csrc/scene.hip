// Scene upload: packs the caller's node arrays into the coalesced device
// layout used by the LoD and splatting kernels, and precomputes theta and
// log(theta) per Gaussian (Section 4.2: log theta is computed once, offline).
#include <cstdlib>
#include <cstring>

#include "vy_common.hpp"

namespace {

__global__ __launch_bounds__(256) void pack_lod(int64_t n, const int32_t* __restrict__ parent,
                                                const int32_t* __restrict__ first_child,
                                                const int32_t* __restrict__ child_count,
                                                const float* __restrict__ lo, const float* __restrict__ hi,
                                                float4* __restrict__ lod, int32_t* __restrict__ ccount) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    lod[2 * i + 0] = make_float4(lo[3 * i], lo[3 * i + 1], lo[3 * i + 2], __int_as_float(first_child[i]));
    lod[2 * i + 1] = make_float4(hi[3 * i], hi[3 * i + 1], hi[3 * i + 2], __int_as_float(parent[i]));
    ccount[i] = first_child[i] >= 0 ? child_count[i] : 0;
  }
}

__global__ __launch_bounds__(256) void pack_gauss(int64_t n, const float* __restrict__ mean,
                                                  const float* __restrict__ ls, const float* __restrict__ quat,
                                                  const float* __restrict__ logit, float4* __restrict__ gauss) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float o = logit[i];
    // theta = 1 / (1 + e^-o); log theta = -log(1 + e^-o), evaluated without overflow
    const float e = expf(-fabsf(o));
    const float theta = o >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
    const float log_theta = o >= 0.f ? -log1pf(e) : o - log1pf(e);
    const float qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2], qz = quat[4 * i + 3];
    const float qn = 1.f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    gauss[3 * i + 0] = make_float4(mean[3 * i], mean[3 * i + 1], mean[3 * i + 2], log_theta);
    gauss[3 * i + 1] = make_float4(expf(ls[3 * i]), expf(ls[3 * i + 1]), expf(ls[3 * i + 2]), theta);
    gauss[3 * i + 2] = make_float4(qw * qn, qx * qn, qy * qn, qz * qn);
  }
}

// Tree depth by pointer jumping: anc[i] is an ancestor of i at distance d[i]
// (anc = -1 once d[i] is the full depth); every round doubles the distance.
__global__ __launch_bounds__(256) void depth_init(int64_t n, const int32_t* __restrict__ parent, int32_t* anc,
                                                  int32_t* d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = parent[i];
    anc[i] = (p >= 0 && p < n) ? p : -1;
    d[i] = (p >= 0 && p < n) ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void depth_jump(int64_t n, const int32_t* __restrict__ anc_in,
                                                  const int32_t* __restrict__ d_in, int32_t* __restrict__ anc_out,
                                                  int32_t* __restrict__ d_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = anc_in[i];
    if (a >= 0) {
      anc_out[i] = anc_in[a];
      d_out[i] = d_in[i] + d_in[a];
    } else {
      anc_out[i] = -1;
      d_out[i] = d_in[i];
    }
  }
}

__global__ __launch_bounds__(256) void depth_max(int64_t n, const int32_t* __restrict__ anc,
                                                 const int32_t* __restrict__ d, int32_t* out) {
  int32_t m = 0, unresolved = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    m = max(m, d[i]);
    unresolved += anc[i] >= 0 ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = max(m, __shfl_xor(m, o, 64));
    unresolved += __shfl_xor(unresolved, o, 64);
  }
  if (__lane_id() == 0) {
    atomicMax(out, m);
    if (unresolved) atomicAdd(out + 1, unresolved);
  }
}

__global__ __launch_bounds__(256) void scene_validate_k(int64_t n, const float4* __restrict__ lod,
                                                        const int32_t* __restrict__ ccount, int32_t* bad) {
  int32_t nb = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 a = lod[2 * i], b = lod[2 * i + 1];
    const int32_t fc = __float_as_int(a.w), par = __float_as_int(b.w);
    bool ok = true;
    if (i == 0) ok = ok && par == -1;
    else ok = ok && par >= 0 && par < n;
    if (ok && i > 0) {
      const float4 pa = lod[2 * (int64_t)par], pb = lod[2 * (int64_t)par + 1];
      const int32_t pfc = __float_as_int(pa.w), pcc = ccount[par];
      ok = ok && pfc >= 0 && i >= pfc && i < (int64_t)pfc + pcc;
      ok = ok && a.x >= pa.x && a.y >= pa.y && a.z >= pa.z && b.x <= pb.x && b.y <= pb.y && b.z <= pb.z;
    }
    const int32_t cc = ccount[i];
    if (fc >= 0) ok = ok && cc > 0 && (int64_t)fc + cc <= n && fc > i;
    else ok = ok && cc == 0;
    ok = ok && a.x <= b.x && a.y <= b.y && a.z <= b.z;
    if (!ok) ++nb;
  }
  if (nb) atomicAdd(bad, nb);
}

}  // namespace

using namespace vy;

extern "C" {

size_t vy_scene_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return (size_t)n * (32 + 4 + 48) + 4 * 256 + 256;  // the 48-byte records double as 4 int scratch arrays
}

int vy_scene_upload(const vy_scene_desc* d, void* ws, size_t ws_bytes, void* stream, vy_scene** out) {
  if (!d || !ws || !out) return fail(VY_ERR_ARG, "vy_scene_upload: NULL argument");
  if (d->n_nodes < 1 || d->n_nodes >= (int64_t(1) << 31))
    return fail(VY_ERR_ARG, "vy_scene_upload: n_nodes %lld out of range", (long long)d->n_nodes);
  if (!d->parent || !d->first_child || !d->child_count || !d->aabb_lo || !d->aabb_hi || !d->mean ||
      !d->log_scale || !d->quat || !d->opacity_logit || !d->sh)
    return fail(VY_ERR_ARG, "vy_scene_upload: NULL array in desc");
  if (ws_bytes < vy_scene_workspace_bytes(d->n_nodes))
    return fail(VY_ERR_ARG, "vy_scene_upload: workspace %zu < %zu bytes", ws_bytes,
                vy_scene_workspace_bytes(d->n_nodes));
  Scene* s = (Scene*)calloc(1, sizeof(Scene));
  if (!s) return fail(VY_ERR_ARG, "vy_scene_upload: out of host memory");
  Carver c(ws, ws_bytes);
  s->magic = kSceneMagic;
  s->n = d->n_nodes;
  s->lod = c.take<float4>(2 * (size_t)s->n);
  s->ccount = c.take<int32_t>(s->n);
  s->gauss = c.take<float4>(3 * (size_t)s->n);
  s->scratch = c.take<int32_t>(64);
  s->sh = d->sh;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)((s->n + 255) / 256 < 8192 ? (s->n + 255) / 256 : 8192);
  int rc = VY_OK;
  int32_t hd[2] = {0, 0};
  do {
    pack_lod<<<blocks, 256, 0, st>>>(s->n, d->parent, d->first_child, d->child_count, d->aabb_lo, d->aabb_hi,
                                     s->lod, s->ccount);
    // the Gaussian records' memory is scratch for the depth computation until pack_gauss
    int32_t* scr = reinterpret_cast<int32_t*>(s->gauss);
    int32_t *anc0 = scr, *d0 = scr + s->n, *anc1 = scr + 2 * s->n, *d1 = scr + 3 * s->n;
    depth_init<<<blocks, 256, 0, st>>>(s->n, d->parent, anc0, d0);
    for (int r = 0; r < 10; ++r) {
      depth_jump<<<blocks, 256, 0, st>>>(s->n, anc0, d0, anc1, d1);
      int32_t* t = anc0; anc0 = anc1; anc1 = t;
      t = d0; d0 = d1; d1 = t;
    }
    if (hipMemsetAsync(s->scratch, 0, 2 * sizeof(int32_t), st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    depth_max<<<blocks < 1024 ? blocks : 1024, 256, 0, st>>>(s->n, anc0, d0, s->scratch);
    if (hipMemcpyAsync(hd, s->scratch, sizeof(hd), hipMemcpyDeviceToHost, st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    pack_gauss<<<blocks, 256, 0, st>>>(s->n, d->mean, d->log_scale, d->quat, d->opacity_logit, s->gauss);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) { rc = VY_ERR_HIP; break; }
  } while (0);
  if (rc != VY_OK) {
    free(s);
    return fail(rc, "vy_scene_upload: HIP failure while packing the scene");
  }
  if (hd[1] != 0) {
    free(s);
    return fail(VY_ERR_ARG, "vy_scene_upload: parent links do not form a tree of depth < 1024");
  }
  s->levels = hd[0] + 1;
  *out = (vy_scene*)s;
  return VY_OK;
}

int vy_scene_update_gaussians(vy_scene* scene, const float* mean, const float* log_scale, const float* quat,
                              const float* opacity_logit, const float* sh, void* stream) {
  Scene* s = (Scene*)scene;
  if (!s || s->magic != kSceneMagic || !mean || !log_scale || !quat || !opacity_logit || !sh)
    return fail(VY_ERR_ARG, "vy_scene_update_gaussians: bad argument");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)((s->n + 255) / 256 < 8192 ? (s->n + 255) / 256 : 8192);
  pack_gauss<<<blocks, 256, 0, st>>>(s->n, mean, log_scale, quat, opacity_logit, s->gauss);
  VY_LAUNCHED();
  s->sh = sh;
  ++s->params_version;
  return VY_OK;
}

int vy_scene_validate(const vy_scene* scene, int64_t* n_bad, void* stream) {
  const Scene* s = (const Scene*)scene;
  if (!s || s->magic != kSceneMagic || !n_bad) return fail(VY_ERR_ARG, "vy_scene_validate: bad argument");
  hipStream_t st = (hipStream_t)stream;
  VY_HIP(hipMemsetAsync(s->scratch, 0, sizeof(int32_t), st));
  const int64_t blocks = (s->n + 255) / 256 < 4096 ? (s->n + 255) / 256 : 4096;
  scene_validate_k<<<(int)blocks, 256, 0, st>>>(s->n, s->lod, s->ccount, s->scratch);
  VY_LAUNCHED();
  int32_t h = 0;
  VY_HIP(hipMemcpyAsync(&h, s->scratch, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  VY_HIP(hipStreamSynchronize(st));
  *n_bad = h;
  return VY_OK;
}

int64_t vy_scene_num_nodes(const vy_scene* scene) {
  const Scene* s = (const Scene*)scene;
  return (s && s->magic == kSceneMagic) ? s->n : -1;
}

int vy_scene_free(vy_scene* scene) {
  Scene* s = (Scene*)scene;
  if (!s) return VY_OK;
  if (s->magic != kSceneMagic) return fail(VY_ERR_ARG, "vy_scene_free: not a scene");
  s->magic = 0;
  delete s->part;
  free(s);
  return VY_OK;
}

}  // extern "C"
