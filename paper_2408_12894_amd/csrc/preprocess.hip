// Preprocess: selection (eq. 6), activation (eq. 4), projection (eq. 1 and EWA), culling,
// tile footprint (tiles counted row by row, see project.h), depth key and SH colour, one
// thread per candidate Gaussian.
//
// Memory: one pass over the attributes (12 + 12 + 16 + 4 + 192 bytes per Gaussian, the SH
// row read as 12 dwordx4 loads), 80 bytes written per visible Gaussian (128 when the render
// keeps the backward's state: the colour Jacobian below). The projection runs in FP64
// (see project.h); mu' is stored as its FP32 rounding plus a bf16 residual so that the blend
// kernels can form pixel offsets to better than 1e-6 px. Rejected candidates stop
// after reading the mean (selection) or the mean and logit (near-plane / opacity culls).
#include "project.h"

namespace flod {

// JAC (renders that keep the backward's state): also the colour's Jacobian in the view
// direction and the colours before the clamp, so that the preprocess backward needs no SH
// coefficients (reading 48 bytes per Gaussian instead of 192).
template <bool JAC>
__global__ __launch_bounds__(kBlock) void k_preprocess(PreParams p, PreOut o) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool vis = false;
  bool selected = false;
  int lvl = 0;
  if (i < p.n_total) {
    lvl = level_of(p, i);
    const DevLevel L = level_at(p, lvl);
    const int64_t j = i - L.offset;
    const float m0 = L.means[j * 3 + 0], m1 = L.means[j * 3 + 1], m2 = L.means[j * 3 + 2];
    selected = true;
    if (p.select) {
      float d2 = dist2(m0, m1, m2, p.centre);
      selected = (L.lo2 <= d2) && (d2 < L.hi2);
    }
    uint32_t tiles = 0;
    if (selected) {
      Proj pr;
      view_transform(p.cam, m0, m1, m2, pr);
      const float logit = L.logits[j];
      if (pr.tz > kNearZD && !(logit < p.logit_min)) {
        float ls[3] = {L.log_scales[j * 3 + 0], L.log_scales[j * 3 + 1], L.log_scales[j * 3 + 2]};
        const float4 q4 = reinterpret_cast<const float4 *>(L.quats)[j];
        float q[4] = {q4.x, q4.y, q4.z, q4.w};
        bool ok = project_cov(p.cam, ls, q, L.s_min, pr);
        if (ok && pr.det > 0.0) {
          const float hx = (float)pr.mx, hy = (float)pr.my;
          const float ca = (float)pr.ca, cb = (float)pr.cb, cc = (float)pr.cc;
          Footprint fp;
          uint32_t rx0 = 0xFFFFu, rx1 = 0u;
          const float qg = support_q(logit);
          if (footprint(hx, hy, ca, cb, cc, support_span(qg), p.cam.tiles_y, fp)) {
            for (int ty = fp.ty0; ty <= fp.ty1; ++ty) {
              int tx0, tx1;
              if (row_span(fp, ty, p.cam.tiles_x, tx0, tx1)) {
                tiles += (uint32_t)(tx1 - tx0 + 1);
                rx0 = min(rx0, (uint32_t)tx0);
                rx1 = max(rx1, (uint32_t)tx1);
              }
            }
          }
          if (tiles > 0) {
            vis = true;
            // colour from SH (not on the key path: contraction allowed via fmaf)
            float dx = m0 - p.cam.campos[0], dy = m1 - p.cam.campos[1], dz = m2 - p.cam.campos[2];
            float inv = 1.0f / sqrtf((dx * dx + dy * dy) + dz * dz);
            // the basis before the SH loads for the colour alone, after them with the Jacobian
            // (formed before them, the Jacobian variant measured 3 us slower at 1080p / 1M)
            float Y[16];
            if (!JAC) sh_basis(p.sh_degree, dx * inv, dy * inv, dz * inv, Y);
            const float4 *shv = reinterpret_cast<const float4 *>(L.sh + j * (FLOD_SH_COEFFS * 3));
            const int nk = (p.sh_degree + 1) * (p.sh_degree + 1);
            const int nv4 = (nk * 3 + 3) / 4;
            float sh[48];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
              if (k < nv4) {
                float4 v = shv[k];
                sh[4 * k + 0] = v.x; sh[4 * k + 1] = v.y; sh[4 * k + 2] = v.z; sh[4 * k + 3] = v.w;
              }
            }
            float col[3];
            if (JAC) {
              // the same colours, with J[ch][a] = sum_k sh[k][ch] dY_k / dd_a (d the unit view
              // direction) and the colours before the clamp stored for the backward
              float Gx[16], Gy[16], Gz[16];
              sh_basis(p.sh_degree, dx * inv, dy * inv, dz * inv, Y);
              sh_basis_grad(p.sh_degree, dx * inv, dy * inv, dz * inv, Gx, Gy, Gz);
              float pre[3], J[9];
#pragma unroll
              for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k)
                  if (k < nk) {
                    acc = fmaf(sh[k * 3 + ch], Y[k], acc);
                    jx = fmaf(sh[k * 3 + ch], Gx[k], jx);
                    jy = fmaf(sh[k * 3 + ch], Gy[k], jy);
                    jz = fmaf(sh[k * 3 + ch], Gz[k], jz);
                  }
                pre[ch] = acc + 0.5f;
                col[ch] = fmaxf(pre[ch], 0.0f);
                J[ch * 3 + 0] = jx; J[ch * 3 + 1] = jy; J[ch * 3 + 2] = jz;
              }
              // three planes of n_total float4 (each store instruction writes consecutive float4)
              o.shjac[i] = make_float4(J[0], J[1], J[2], J[3]);
              o.shjac[p.n_total + i] = make_float4(J[4], J[5], J[6], J[7]);
              o.shjac[2 * p.n_total + i] = make_float4(J[8], pre[0], pre[1], pre[2]);
            } else {
#pragma unroll
              for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k)
                  if (k < nk) acc = fmaf(sh[k * 3 + ch], Y[k], acc);
                col[ch] = fmaxf(acc + 0.5f, 0.0f);
              }
            }
            const float opac = 1.0f / (1.0f + __expf(-logit));
            o.xyab[i] = make_float4(hx, hy, ca, cb);
            o.cop[i] = make_float4(cc, opac, col[0], col[1]);
            o.blue[i] = make_float2(col[2], __uint_as_float(pack_mu_lo(pr.mx, pr.my, hx, hy)));
            o.depth[i] = __float_as_uint((float)pr.tz);
            o.bin[2 * i] = make_float4(hx, hy, ca, cb);
            o.bin[2 * i + 1] = make_float4(cc, qg, __uint_as_float(rx0 | ((uint32_t)fp.ty0 << 16)),
                                           __uint_as_float(rx1 | ((uint32_t)fp.ty1 << 16)));
          }
        }
      }
    }
    o.tiles[i] = tiles;
    if (!vis) o.depth[i] = kDepthNone;   // the depth sort's first pass skips it
  }
  if (o.zero_sums && threadIdx.x == 0) o.zero_sums[blockIdx.x] = 0u;
  // per-level selected counts, aggregated per wave
  if (o.n_selected) {
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < p.n_levels; ++k) {
      unsigned long long m = __ballot(selected && lvl == k);
      if (lane == 0 && m) atomicAdd(&o.n_selected[k], (unsigned long long)__popcll(m));
    }
  }
  int cnt = __syncthreads_count(vis);
  if (threadIdx.x == 0) o.block_vis[blockIdx.x] = (uint32_t)cnt;
}

hipError_t launch_preprocess(const PreParams &p, const PreOut &o, hipStream_t s) {
  if (p.n_total <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((p.n_total + kBlock - 1) / kBlock);
  if (o.shjac)
    hipLaunchKernelGGL(k_preprocess<true>, dim3(grid), dim3(kBlock), 0, s, p, o);
  else
    hipLaunchKernelGGL(k_preprocess<false>, dim3(grid), dim3(kBlock), 0, s, p, o);
  return hipGetLastError();
}

}  // namespace flod
