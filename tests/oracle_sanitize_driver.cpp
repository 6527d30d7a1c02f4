// Drives the oracle's C entry points on small synthetic inputs so that a build
// with AddressSanitizer and UndefinedBehaviorSanitizer sees every stage:
// measurement, sequences (real, complex and bicomplex seeds), state-loaded
// steps, fusion, raycast, ICP objective, relocalisation objective and the
// surfel front end.  Built and run by test_oracle_sanitizers.py; exits 0 when
// every call returned and the results are finite.
#include "../oracle/xslam_oracle.cpp"

#include <cstdio>

namespace {

constexpr int kW = 32, kH = 24, kDim = 24;

OrcConfig small_config() {
  OrcConfig c{};
  c.width = kW; c.height = kH;
  c.fx = 28.0; c.fy = 28.0; c.cx = 15.5; c.cy = 11.5;
  c.dim[0] = c.dim[1] = c.dim[2] = kDim;
  c.voxel = 0.04; c.trunc = 0.12; c.wcap = 64.0;
  c.iters[0] = 3; c.iters[1] = 2; c.iters[2] = 0;
  c.dgate = 0.1; c.agate_deg = 20.0;
  c.level_w[0] = c.level_w[1] = c.level_w[2] = 1.0;
  c.disc_delta = 0.1;
  c.bilateral_radius = 2; c.sigma_px = 4.5; c.sigma_m = 0.03;
  c.near_m = 0.1;
  c.pf_d_depth = 0.05; c.pf_d_norm_deg = 30.0; c.pf_d_dist = 0.05; c.pf_sigma = 0.02; c.pf_c_stable = 0.0;
  c.pf_capacity = 8 * kW * kH;
  return c;
}

// three planes seen from a camera at z = -1: a box corner, with a hole
void depth_frame(int k, double* d) {
  for (int y = 0; y < kH; ++y)
    for (int x = 0; x < kW; ++x) {
      const double rx = (x - 15.5) / 28.0, ry = (y - 11.5) / 28.0;
      double z = 1.0 / (1.0 - 0.3 * rx - 0.002 * k);
      if (x >= kW / 2) z = 0.9 / (1.0 - 0.4 * ry);
      if (y >= 2 * kH / 3 && x < kW / 2) z = 1.05 / (1.0 + 0.3 * rx);
      if (x == 3 && y == 4) z = 0.0;
      d[y * kW + x] = z;
    }
}

bool finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

int main() {
  const OrcConfig c = small_config();
  const size_t npx = size_t(kW) * kH, nv = size_t(kDim) * kDim * kDim;
  const int nf = 3;
  std::vector<double> depths(nf * npx), dots(nf * npx, 0.01);
  for (int k = 0; k < nf; ++k) depth_frame(k, depths.data() + k * npx);
  double T0[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 1};
  bool ok = true;
  const OrcSeed seeds[3] = {{0, -1, -1, 0.0}, {1, 3, -1, 1e-20}, {2, 0, 13, 1e-20}};
  for (const OrcSeed& s : seeds) {
    const int nc = s.kind == 0 ? 1 : s.kind == 1 ? 2 : 4;
    std::vector<double> poses(nf * 16 * nc), stats(nf * 6), F(nv * nc), Wt(nv * nc);
    orc_run_sequence(&c, &s, nf, depths.data(), dots.data(), T0, poses.data(), stats.data(), F.data(), Wt.data(),
                     nullptr, nullptr);
    ok = ok && finite(poses.data(), poses.size()) && finite(F.data(), F.size());
    // measurement and raycast of the final volume
    size_t tot = npx + npx / 4 + npx / 16;
    std::vector<double> Dm(tot * nc), Vm(tot * 3 * nc), Nm(tot * 3 * nc);
    std::vector<uint8_t> vm(tot);
    orc_measure(&c, &s, depths.data(), dots.data(), Dm.data(), Vm.data(), Nm.data(), vm.data());
    std::vector<double> V(npx * 3 * nc), N(npx * 3 * nc), Z(npx);
    std::vector<uint8_t> valid(npx);
    orc_raycast(&c, &s, F.data(), Wt.data(), poses.data() + (nf - 1) * 16 * nc, nullptr, 0, V.data(), N.data(),
                Z.data(), valid.data(), nullptr, nullptr);
    ok = ok && finite(V.data(), V.size()) && finite(Dm.data(), Dm.size());
    // surfel front end
    std::vector<double> pposes(nf * 16 * nc), pstats(nf * 6);
    std::vector<int64_t> pf(nf * 3);
    const size_t cap = size_t(c.pf_capacity);
    std::vector<double> sv(cap * 3 * nc), sn(cap * 3 * nc), sr(cap * nc), sc(cap * nc);
    std::vector<int32_t> st(cap);
    int64_t count = 0;
    orc_pf_run_sequence(&c, &s, nf, depths.data(), dots.data(), T0, pposes.data(), pstats.data(), pf.data(),
                        sv.data(), sn.data(), sr.data(), sc.data(), st.data(), &count);
    ok = ok && count > 0 && finite(sv.data(), size_t(count) * 3 * nc);
  }
  // real-run objectives: ICP (held and through) and relocalisation
  {
    const OrcSeed s{0, -1, -1, 0.0};
    std::vector<double> poses(nf * 16), stats(nf * 6), F(nv), Wt(nv);
    orc_run_sequence(&c, &s, nf, depths.data(), nullptr, T0, poses.data(), stats.data(), F.data(), Wt.data(),
                     nullptr, nullptr);
    size_t tot = npx + npx / 4 + npx / 16;
    std::vector<double> Dm(tot), Vm(tot * 3), Nm(tot * 3);
    std::vector<uint8_t> vm(tot);
    orc_measure(&c, &s, depths.data() + (nf - 1) * npx, nullptr, Dm.data(), Vm.data(), Nm.data(), vm.data());
    std::vector<double> V(npx * 3), N(npx * 3), Z(npx);
    std::vector<uint8_t> valid(npx);
    orc_raycast(&c, &s, F.data(), Wt.data(), poses.data() + (nf - 2) * 16, nullptr, 0, V.data(), N.data(), Z.data(),
                valid.data(), nullptr, nullptr);
    double out[29];
    for (int through = 0; through < 2; ++through) {
      orc_icp_energy(&c, 0, Vm.data(), Nm.data(), vm.data(), V.data(), N.data(), Z.data(), valid.data(),
                     poses.data() + (nf - 2) * 16, poses.data() + (nf - 1) * 16, through, 2, out);
      ok = ok && finite(out, 29);
    }
    orc_reloc_energy(&c, F.data(), Wt.data(), Dm.data(), poses.data() + (nf - 1) * 16, 2, out);
    ok = ok && finite(out, 29);
  }
  std::printf("%s\n", ok ? "sanitized oracle run: ok" : "sanitized oracle run: non-finite result");
  return ok ? 0 : 1;
}
