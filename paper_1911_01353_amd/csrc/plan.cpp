// Plan: the (zbar, w) lattice, per-template half-widths, width groups and the
// byte layout of the template bank. Host code only; no HIP calls.
//
// Lattice and response follow the paper's section "Implementation" (filters
// indexed by z = fdot T^2 and w = fddot T^3, one z set per w, Figure 2). The
// half-width rule: the template's tone sweeps at most |zbar|/2 + |w|/12 bins
// away from the trial frequency over the observation (end points of the
// centred sweep -w/24 + zbar s + w s^2/2 on s in [-1/2, 1/2]); h = ceil of that
// plus a margin.
#include <algorithm>
#include <cmath>
#include <map>

#include "jerk_internal.h"

namespace jerk {

bool seg_len_supported(int32_t s) { return s == 512 || s == 1024 || s == 2048 || s == 4096; }

namespace {

// 16-point Gauss-Legendre rule on [-1, 1] by Newton's method on P_16.
void gauss_legendre16(double* x, double* w) {
  const int n = 16;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // recompute the derivative at the converged root for the weight
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wt;
    w[n - 1 - i] = wt;
  }
}

// Segment length before autotuning: 1024 (with 16 elements per thread the
// fastest single choice on gfx950 for searches without a plane, and within a
// few percent of the per-group best for plane-writing ones, where the
// autotuner picks 512 for narrow and 2048 for wide groups), longer only for
// wider templates.
int32_t default_seg_len(int32_t taps) {
  const int32_t cand[3] = {1024, 2048, 4096};
  for (int32_t s : cand)
    if (s >= 2 * taps) return s;
  return 4096;
}

// Elements per thread of the default FFT kernel variant of a segment length.
int32_t default_ept(int32_t seg_len) { return seg_len == 512 ? 8 : 16; }

// Templates per workgroup before autotuning: the largest of 64, 32, 16, 8 whose
// launch over the whole group still has 4096 workgroups, else 4. Larger blocks
// let each segment's forward transform and spectrum reads serve more templates
// (64 against 16 on the 2^22-bin search: 3.5% faster writing the plane, 7.5%
// returning peaks); small searches need the smaller blocks to fill the device
// (2^15 bins: 24.6 us at 4 per block against 63 us at 16).
int32_t default_tpb(int64_t nbins, int32_t seg_len, int32_t taps, int64_t members) {
  const int64_t n_seg = (nbins + (seg_len - taps + 1) - 1) / (seg_len - taps + 1);
  for (int32_t tpb : {64, 32, 16, 8})
    if (n_seg * ((members + tpb - 1) / tpb) >= 4096) return tpb;
  return 4;
}

// Largest group width the split-BF16 path is chosen for under JERK_PATH_AUTO
// (the FFT path's cost per output is nearly independent of the width, the
// direct correlation's grows linearly with it).
constexpr int32_t kAutoGemmMaxTaps = 96;
// Widest group the MFMA kernels accept.
constexpr int32_t kGemmMaxTaps = 512;

}  // namespace

void plan_layout(Plan& p) {
  size_t off = 0;
  p.off_members = off;
  off = align_up(off + sizeof(int32_t) * (size_t)p.T);
  for (int i = 0; i < 4; ++i) {
    p.off_tw[i] = off;
    off = align_up(off + (size_t)(512 << i) * 8);
  }
  int32_t first = 0;
  for (auto& g : p.groups) {
    g.first_member = first;
    first += (int32_t)g.members.size();
  }
  for (auto& g : p.groups) {
    g.off_taps = off;
    off = align_up(off + g.members.size() * 2 * (size_t)g.taps * 16);
  }
  for (auto& g : p.groups) {
    g.off_fft = 0;
    g.off_gemm = 0;
    g.gemm_bytes = 0;
    if (g.path == JERK_PATH_FFT_FP32) {
      g.off_fft = off;
      off = align_up(off + g.members.size() * 2 * (size_t)g.seg_len * 8);
    } else {
      g.off_gemm = off;
      g.gemm_bytes = gemm_bank_bytes((int32_t)g.members.size(), g.taps, g.path);
      off = align_up(off + g.gemm_bytes);
    }
  }
  p.bank_bytes = off;
}

void plan_build(Plan& p, const jerk_plan_desc& d) {
  require(d.nbins >= 1, JERK_EINVAL, "nbins must be >= 1");
  require(std::isfinite(d.zmax) && d.zmax >= 0.0, JERK_EINVAL, "zmax must be finite and >= 0");
  require(std::isfinite(d.wmax) && d.wmax >= 0.0, JERK_EINVAL, "wmax must be finite and >= 0");
  require(std::isfinite(d.dz) && d.dz > 0.0, JERK_EINVAL, "dz must be > 0");
  require(std::isfinite(d.dw) && (d.dw > 0.0 || (d.dw == 0.0 && d.wmax == 0.0)), JERK_EINVAL,
          "dw must be > 0 (or 0 with wmax == 0)");
  require(d.numbetween == 2, JERK_EINVAL, "numbetween must be 2 (half-bin spacing)");
  require(d.margin_bins >= 0 && d.margin_bins <= 256, JERK_EINVAL, "margin_bins must be in [0, 256]");
  require(d.path >= JERK_PATH_FFT_FP32 && d.path <= JERK_PATH_AUTO, JERK_EINVAL, "unknown path");
  require(d.seg_len == 0 || seg_len_supported(d.seg_len), JERK_EINVAL,
          "seg_len must be 0, 512, 1024, 2048 or 4096");
  require(d.templates_per_block >= 0 && d.templates_per_block <= 64, JERK_EINVAL,
          "templates_per_block must be in [0, 64]");
  require(d.tap_quantum == 0 || (d.tap_quantum >= 16 && d.tap_quantum <= 512 && d.tap_quantum % 16 == 0),
          JERK_EINVAL, "tap_quantum must be 0 or a multiple of 16 in [16, 512]");
  require(d.flags == 0, JERK_EINVAL, "flags must be 0");
  const double nz_real = 2.0 * d.zmax / d.dz;
  const double nw_real = d.dw > 0.0 ? d.wmax / d.dw : 0.0;
  require(nz_real < 1e6 && nw_real < 1e6, JERK_EINVAL, "lattice too large");

  p.desc = d;
  p.n_z = (int32_t)std::floor(nz_real + 1e-9) + 1;
  p.J = d.dw > 0.0 ? (int32_t)std::floor(nw_real + 1e-9) : 0;
  p.n_w = 2 * p.J + 1;
  require((int64_t)p.n_z * p.n_w <= (1 << 24), JERK_EINVAL, "more than 2^24 templates");
  p.T = p.n_z * p.n_w;
  p.zbar.resize(p.T);
  p.w.resize(p.T);
  p.half.resize(p.T);
  p.group_of.resize(p.T);
  p.slot.resize(p.T);
  const int32_t quantum = d.tap_quantum ? d.tap_quantum : 16;
  std::map<int32_t, std::vector<int32_t>> by_width;
  p.max_taps = 0;
  for (int32_t t = 0; t < p.T; ++t) {
    const int32_t i = t % p.n_z, j = t / p.n_z;
    const double zb = -d.zmax + i * d.dz;
    const double ww = (j - p.J) * d.dw;
    const double fmax = std::fabs(zb) / 2.0 + std::fabs(ww) / 12.0;
    const int32_t h = (int32_t)std::ceil(fmax) + d.margin_bins;
    require(h >= 1, JERK_EINVAL, "template half-width is 0 (margin_bins = 0 with zbar = w = 0)");
    p.zbar[t] = zb;
    p.w[t] = ww;
    p.half[t] = h;
    p.max_taps = std::max(p.max_taps, 2 * h);
    const int32_t kg = (2 * h + quantum - 1) / quantum * quantum;
    by_width[kg].push_back(t);
  }
  p.groups.clear();
  for (auto& kv : by_width) {
    Group g;
    g.taps = kv.first;
    g.members = kv.second;
    g.seg_len = d.seg_len ? d.seg_len : default_seg_len(g.taps);
    require(g.taps <= 2048, JERK_EUNSUPPORTED, "template wider than 2048 taps");
    require(g.seg_len >= 2 * g.taps, JERK_EINVAL, "seg_len must be at least twice the widest group's taps");
    g.tpb = d.templates_per_block ? d.templates_per_block
                                  : default_tpb(d.nbins, g.seg_len, g.taps, (int64_t)g.members.size());
    g.ept = default_ept(g.seg_len);
    if (d.path == JERK_PATH_AUTO) {
      g.path = g.taps <= kAutoGemmMaxTaps ? JERK_PATH_GEMM_SPLIT_BF16 : JERK_PATH_FFT_FP32;
    } else {
      g.path = d.path;
      if (d.path != JERK_PATH_FFT_FP32)
        require(g.taps <= kGemmMaxTaps, JERK_EUNSUPPORTED,
                "MFMA paths support templates up to 512 taps; use the FFT or AUTO path");
    }
    const int32_t gi = (int32_t)p.groups.size();
    for (size_t s = 0; s < g.members.size(); ++s) {
      p.group_of[g.members[s]] = gi;
      p.slot[g.members[s]] = (int32_t)s;
    }
    p.groups.push_back(std::move(g));
  }
  gauss_legendre16(p.gl_x, p.gl_w);
  plan_layout(p);
}

}  // namespace jerk
