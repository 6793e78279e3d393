// C ABI of the online hyper-reduced solve: artifact loading, state
// management and the per-step entry points declared in podecm.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "rom_fused.h"
#include "rom_staged.h"

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
  if (hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T)) != hipSuccess) return ROM_EHIP;
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return ROM_EHIP;
  return ROM_OK;
}

void release(rom_model* h) {
  if (!h) return;
  for (int i = 0; i < 2 * h->cap; ++i) (void)hipEventDestroy(h->ev[i]);
  free(h->ev);
  if (h->aux) {
    (void)hipStreamSynchronize(h->aux);
    (void)hipStreamDestroy(h->aux);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  (void)hipFree(h->w);
  (void)hipFree(h->Gt);
  (void)hipFree(h->Gq);
  (void)hipFree(h->Gd);
  (void)hipFree(h->Gq32);
  (void)hipFree(h->Gq16);
  (void)hipFree(h->phase);
  delete h;
}

}  // namespace

int rom_timing_mark(rom_model* h, int stop, hipStream_t s) {
  if (!h->timing) return ROM_OK;
  if (!stop && h->nev == h->cap) {
    const int ncap = h->cap ? 2 * h->cap : 256;
    hipEvent_t* ev = static_cast<hipEvent_t*>(realloc(h->ev, sizeof(hipEvent_t) * 2 * ncap));
    if (!ev) return ROM_EINVAL;
    h->ev = ev;
    for (int i = 2 * h->cap; i < 2 * ncap; ++i)
      if (hipEventCreate(&h->ev[i]) != hipSuccess) return ROM_EHIP;
    h->cap = ncap;
  }
  const int slot = stop ? 2 * (h->nev - 1) + 1 : 2 * h->nev;
  if (hipEventRecord(h->ev[slot], s) != hipSuccess) return ROM_EHIP;
  if (!stop) ++h->nev;
  return ROM_OK;
}

extern "C" {

int rom_timing_enable(rom_handle h, int enable) {
  if (!h) return ROM_EINVAL;
  h->timing = enable ? 1 : 0;
  h->nev = 0;
  return ROM_OK;
}

int rom_timing_read(rom_handle h, double* total_ms, int64_t* launches) {
  if (!h || !total_ms || !launches) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  double tot = 0.0;
  for (int i = 0; i < h->nev; ++i) {
    if (hipEventSynchronize(h->ev[2 * i + 1]) != hipSuccess) return ROM_EHIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) != hipSuccess) return ROM_EHIP;
    tot += ms;
  }
  *total_ms = tot;
  *launches = h->nev;
  return ROM_OK;
}

int rom_default_opts(rom_opts* o) {
  if (!o) return ROM_EINVAL;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iter = 15;
  o->fixed_iters = 0;
  o->commit = 1;
  o->contraction = ROM_DT_F64;
  o->mode = ROM_MODE_STAGED;
  o->warm_start = ROM_WARM_PREV;
  o->split = -1;
  o->grid_per_cu = 0;
  o->max_substeps = 0;
  o->phased_evals = 0;
  o->phased_early = 0;
  o->abar_f64 = 0;
  o->mlp = nullptr;
  o->active = nullptr;
  return ROM_OK;
}

int rom_load(const void* blob, size_t bytes, int device, rom_handle* out) {
  if (!blob || !out) return ROM_EINVAL;
  *out = nullptr;
  const unsigned char* b = static_cast<const unsigned char*>(blob);
  if (bytes < 256 || memcmp(b, "PODECMR1", 8) != 0) return ROM_EFORMAT;
  uint32_t hdr[6];
  memcpy(hdr, b + 8, sizeof(hdr));
  if (hdr[0] != 1 && hdr[0] != 2) return ROM_EVERSION;
  const bool two = hdr[0] == 2;  // version 2: a second phase and the phase of every point
  const int n = (int)hdr[1], m = (int)hdr[2], c = (int)hdr[3], kind = (int)hdr[4], n_mu = (int)hdr[5];
  if (n < 1 || n > ROM_NMAX - 5 || m < 1 || m > (1 << 24) || c < 1 || c > 12) return ROM_EFORMAT;
  if (!((kind == 0 && c == 2 && n_mu == 2) || (kind == 1 && c == 12 && n_mu == 8) || (kind == 2 && c == 1 && n_mu == 1)))
    return ROM_EFORMAT;
  double par[7];
  memcpy(par, b + 32, sizeof(par));
  const size_t need = 256 + 8 * ((size_t)m + (size_t)m * 4 * n + (size_t)m * 4 * c + (size_t)m + (two ? (size_t)m : 0));
  if (bytes < need) return ROM_EFORMAT;
  for (int i = 0; i < 7; ++i)
    if (!isfinite(par[i])) return ROM_EFORMAT;
  const double E = par[0], nu = par[1];
  // the parent void radius r0 enters the voids' maps only (kinds 0 and 1)
  if (!(E > 0 && nu > -1 && nu < 0.5 && par[2] > 0 && par[3] >= 0 && (kind == 2 || par[4] > 0) && par[6] > 0))
    return ROM_EFORMAT;
  double par2[4] = {E, nu, par[2], par[3]};
  std::vector<int> phase;
  if (two) {
    memcpy(par2, b + 88, sizeof(par2));
    for (int i = 0; i < 4; ++i)
      if (!isfinite(par2[i])) return ROM_EFORMAT;
    if (!(par2[0] > 0 && par2[1] > -1 && par2[1] < 0.5 && par2[2] > 0 && par2[3] >= 0)) return ROM_EFORMAT;
    const unsigned char* pp = b + 256 + 8 * ((size_t)m + (size_t)m * 4 * n + (size_t)m * 4 * c + (size_t)m);
    phase.resize(m);
    for (int q = 0; q < m; ++q) {
      int64_t v;
      memcpy(&v, pp + 8 * (size_t)q, 8);
      if (v != 0 && v != 1) return ROM_EFORMAT;
      phase[q] = (int)v;
    }
  }
  std::vector<double> w(m), G((size_t)m * 4 * n), Gd((size_t)m * 4 * c);
  const unsigned char* p = b + 256;
  memcpy(w.data(), p, 8 * w.size());
  p += 8 * w.size();
  memcpy(G.data(), p, 8 * G.size());
  p += 8 * G.size();
  memcpy(Gd.data(), p, 8 * Gd.size());
  for (double v : w)
    if (!(v > 0) || !isfinite(v)) return ROM_EFORMAT;
  for (double v : G)
    if (!isfinite(v)) return ROM_EFORMAT;
  for (double v : Gd)
    if (!isfinite(v)) return ROM_EFORMAT;
  // padded width: the fused contraction carries f and C in columns n .. n+4
  const int npad = 16 * rom_fused_tiles(n);
  std::vector<double> Gt((size_t)n * 4 * m), Gq((size_t)m * 4 * npad, 0.0), Gdt((size_t)c * 4 * m);
  std::vector<float> Gq32((size_t)m * 4 * npad, 0.0f);
  std::vector<uint16_t> Gq16((size_t)m * 4 * npad, 0);
  for (int q = 0; q < m; ++q)
    for (int a = 0; a < 4; ++a) {
      for (int i = 0; i < n; ++i) {
        const double v = G[((size_t)q * 4 + a) * n + i];
        Gt[((size_t)i * 4 + a) * m + q] = v;
        Gq[((size_t)q * 4 + a) * npad + i] = v;
        Gq32[((size_t)q * 4 + a) * npad + i] = (float)v;
        Gq16[((size_t)q * 4 + a) * npad + i] = f32_to_bf16_rne((float)v);
      }
      for (int k = 0; k < c; ++k) Gdt[((size_t)k * 4 + a) * m + q] = Gd[((size_t)q * 4 + a) * c + k];
    }
  DeviceGuard guard(device);
  rom_model* h = new rom_model();
  memset(h, 0, sizeof(*h));
  h->device = device;
  h->n = n;
  h->m = m;
  h->c = c;
  h->kind = kind;
  h->n_mu = n_mu;
  h->npad = npad;
  h->E = E;
  h->nu = nu;
  h->sy0 = par[2];
  h->H = par[3];
  h->r0 = par[4];
  h->void_area = par[5];
  h->cell_area = par[6];
  h->mp.G = E / (2.0 * (1.0 + nu));
  h->mp.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  h->mp.K = h->mp.lam + 2.0 * h->mp.G / 3.0;
  h->mp.sy0 = par[2];
  h->mp.H = par[3];
  h->mp2.G = par2[0] / (2.0 * (1.0 + par2[1]));
  h->mp2.lam = par2[0] * par2[1] / ((1.0 + par2[1]) * (1.0 - 2.0 * par2[1]));
  h->mp2.K = h->mp2.lam + 2.0 * h->mp2.G / 3.0;
  h->mp2.sy0 = par2[2];
  h->mp2.H = par2[3];
  int rc = ROM_OK;
  if (two) rc = upload(&h->phase, phase);
  if (rc == ROM_OK && hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    rc = ROM_EHIP;
  if (rc == ROM_OK) rc = upload(&h->w, w);
  if (rc == ROM_OK) rc = upload(&h->Gt, Gt);
  if (rc == ROM_OK) rc = upload(&h->Gq, Gq);
  if (rc == ROM_OK) rc = upload(&h->Gd, Gdt);
  if (rc == ROM_OK) rc = upload(&h->Gq32, Gq32);
  if (rc == ROM_OK) rc = upload(&h->Gq16, Gq16);
  if (rc == ROM_OK) rc = rom_staged_setup();
  if (rc == ROM_OK) rc = rom_fused_setup();
  if (rc == ROM_OK) rc = rom_noalloc_setup(device);  // the static scratch of rom_step_noalloc on this device
  // side stream and events of the phased form (created here, not inside a
  // caller's graph capture)
  if (rc == ROM_OK && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) rc = ROM_EHIP;
  if (rc == ROM_OK && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess) rc = ROM_EHIP;
  if (rc == ROM_OK && hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) rc = ROM_EHIP;
  if (rc != ROM_OK) {
    release(h);
    return rc;
  }
  *out = h;
  return ROM_OK;
}

int rom_load_file(const char* path, int device, rom_handle* out) {
  if (!path || !out) return ROM_EINVAL;
  FILE* fh = fopen(path, "rb");
  if (!fh) return ROM_EINVAL;
  std::vector<unsigned char> buf;
  unsigned char tmp[1 << 16];
  size_t got;
  while ((got = fread(tmp, 1, sizeof(tmp), fh)) > 0) buf.insert(buf.end(), tmp, tmp + got);
  fclose(fh);
  return rom_load(buf.data(), buf.size(), device, out);
}

int rom_free(rom_handle h) {
  if (!h) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  release(h);
  return ROM_OK;
}

int rom_info(rom_handle h, int32_t* n, int32_t* m, int32_t* c, int32_t* n_mu) {
  if (!h) return ROM_EINVAL;
  if (n) *n = h->n;
  if (m) *m = h->m;
  if (c) *c = h->c;
  if (n_mu) *n_mu = h->n_mu;
  return ROM_OK;
}

int rom_state_bytes(rom_handle h, int32_t batch, size_t* bytes) {
  if (!h || !bytes || batch < 0) return ROM_EINVAL;
  *bytes = rom_state_layout(h, (size_t)batch).total;
  return ROM_OK;
}

int rom_state_offsets(rom_handle h, int32_t batch, size_t* offsets) {
  if (!h || !offsets || batch < 0) return ROM_EINVAL;
  const StateLayout L = rom_state_layout(h, (size_t)batch);
  for (int i = 0; i < ROM_NFIELDS; ++i) offsets[i] = L.off[i];
  return ROM_OK;
}

int rom_state_init(rom_handle h, int32_t batch, const double* mu_dev, void* state_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!mu_dev || !state_dev || batch > 65535) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  int rc = rom_launch_state_init(h, batch, mu_dev, state_dev, stream);
  if (rc != ROM_OK) return rc;
  const StateLayout L = rom_state_layout(h, batch);
  int bad = 0;
  if (hipMemcpyAsync(&bad, field<int>(state_dev, L, F_COUNT), sizeof(int), hipMemcpyDeviceToHost, stream) !=
      hipSuccess)
    return ROM_EHIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return ROM_EHIP;
  return bad ? ROM_EINVAL_MU : ROM_OK;
}

int rom_step(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev, const rom_opts* opts,
             int32_t* status_dev, int32_t* iters_dev, double* resnorm_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!Fbar_dev || !state_dev || !status_dev || !iters_dev || !resnorm_dev || batch > 65535) return ROM_EINVAL;
  rom_opts o;
  if (opts)
    o = *opts;
  else
    rom_default_opts(&o);
  if (o.max_iter < 1 || o.max_iter > 1000 || !(o.tol >= 0.0)) return ROM_EINVAL;
  if (o.contraction < ROM_DT_F64 || o.contraction > ROM_DT_BF16) return ROM_EINVAL;
  if (o.abar_f64 != 0 && o.abar_f64 != 1) return ROM_EINVAL;
  if (o.warm_start != ROM_WARM_PREV && o.warm_start != ROM_WARM_MLP) return ROM_EINVAL;
  if (o.warm_start == ROM_WARM_MLP && !o.mlp) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  if (o.grid_per_cu < 0 || o.grid_per_cu > 64) return ROM_EINVAL;
  if (o.max_substeps < 0 || o.max_substeps > ROM_MAX_SUBSTEPS) return ROM_EINVAL;
  if (o.max_substeps > 0 && !o.commit) return ROM_EUNSUPPORTED;  // sub-steps are committed as they converge
  if (o.mode == ROM_MODE_STAGED) {
    if (o.contraction != ROM_DT_F64 || o.warm_start != ROM_WARM_PREV || o.active || o.grid_per_cu ||
        o.max_substeps)
      return ROM_EUNSUPPORTED;
    return rom_launch_step_staged(h, batch, Fbar_dev, state_dev, o, status_dev, iters_dev, resnorm_dev, stream);
  }
  if (o.mode == ROM_MODE_FUSED)
    return rom_launch_step_fused(h, batch, Fbar_dev, state_dev, o, status_dev, iters_dev, resnorm_dev, stream);
  if (o.mode == ROM_MODE_PHASED) {
    if (o.phased_evals < 0 || o.phased_early < -1) return ROM_EINVAL;
    return rom_launch_step_phased(h, batch, Fbar_dev, state_dev, o, status_dev, iters_dev, resnorm_dev, stream);
  }
  return ROM_EINVAL;
}

int rom_step_noalloc(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev, const rom_opts* opts,
                     int32_t* status_dev, int32_t* iters_dev, double* resnorm_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (batch > ROM_NOALLOC_MAX_BATCH) return ROM_ESCRATCH;
  if (!Fbar_dev || !state_dev || !status_dev || !iters_dev || !resnorm_dev) return ROM_EINVAL;
  rom_opts o;
  if (opts)
    o = *opts;
  else
    rom_default_opts(&o);
  if (o.max_iter < 1 || o.max_iter > 1000 || !(o.tol >= 0.0)) return ROM_EINVAL;
  if (o.contraction < ROM_DT_F64 || o.contraction > ROM_DT_BF16) return ROM_EINVAL;
  if (o.abar_f64 != 0 && o.abar_f64 != 1) return ROM_EINVAL;
  if (o.warm_start != ROM_WARM_PREV && o.warm_start != ROM_WARM_MLP) return ROM_EINVAL;
  if (o.warm_start == ROM_WARM_MLP && !o.mlp) return ROM_EINVAL;
  if (o.grid_per_cu < 0 || o.grid_per_cu > 64) return ROM_EINVAL;
  if (o.max_substeps < 0 || o.max_substeps > ROM_MAX_SUBSTEPS) return ROM_EINVAL;
  if (o.max_substeps > 0 && !o.commit) return ROM_EUNSUPPORTED;
  if (o.mode != ROM_MODE_FUSED) return ROM_EUNSUPPORTED;
  DeviceGuard guard(h->device);
  return rom_launch_step_noalloc(h, batch, Fbar_dev, state_dev, o, status_dev, iters_dev, resnorm_dev, stream);
}

int rom_shape_sensitivity(rom_handle h, int32_t batch, const double* Fbar_dev, const void* state_dev,
                          double* dPdmu_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!Fbar_dev || !state_dev || !dPdmu_dev || batch > 65535) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  return rom_launch_shape_sensitivity(h, batch, Fbar_dev, state_dev, dPdmu_dev, stream);
}

int rom_features(rom_handle h, int32_t batch, const double* Fbar_dev, const void* state_dev, float* X_dev,
                 hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!Fbar_dev || !state_dev || !X_dev || batch > 65535) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  return rom_launch_features(h, batch, Fbar_dev, state_dev, X_dev, stream);
}

int rom_warm_samples(rom_handle h, int32_t batch, const void* state_dev, const float* X_feat_dev,
                     const double* r_before_dev, const int32_t* status_dev, float* X_out_dev, float* Y_out_dev,
                     int32_t* count_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!state_dev || !X_feat_dev || !r_before_dev || !status_dev || !X_out_dev || !Y_out_dev || !count_dev ||
      batch > 65535)
    return ROM_EINVAL;
  DeviceGuard guard(h->device);
  return rom_launch_warm_samples(h, batch, state_dev, X_feat_dev, r_before_dev, status_dev, X_out_dev, Y_out_dev,
                                 count_dev, stream);
}

int rom_commit_trial(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev,
                     const int32_t* status_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!Fbar_dev || !state_dev || !status_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  return rom_launch_commit_trial(h, batch, Fbar_dev, state_dev, status_dev, stream);
}

int rom_path_gather(int32_t batch, const double* paths, int32_t max_steps, const int32_t* nsteps,
                    const int32_t* step, double* Fbar, int32_t* active, hipStream_t stream) {
  if (batch < 0 || max_steps < 1) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!paths || !nsteps || !step || !Fbar || !active) return ROM_EINVAL;
  return rom_launch_path_gather(batch, paths, max_steps, nsteps, step, Fbar, active, stream);
}

int rom_path_advance(int32_t batch, const int32_t* active, int32_t* step, hipStream_t stream) {
  if (batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!active || !step) return ROM_EINVAL;
  return rom_launch_path_advance(batch, active, step, stream);
}

int rom_homogenized_stress_tangent(rom_handle h, int32_t batch, const void* state_dev, double* Pbar_dev,
                                   double* Abar_dev, hipStream_t stream) {
  if (!h || batch < 0) return ROM_EINVAL;
  if (batch == 0) return ROM_OK;
  if (!state_dev || !Pbar_dev || !Abar_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  const StateLayout L = rom_state_layout(h, batch);
  void* st = const_cast<void*>(state_dev);
  if (hipMemcpyAsync(Pbar_dev, field<double>(st, L, F_PBAR), (size_t)batch * 4 * 8, hipMemcpyDeviceToDevice,
                     stream) != hipSuccess)
    return ROM_EHIP;
  if (hipMemcpyAsync(Abar_dev, field<double>(st, L, F_ABAR), (size_t)batch * 16 * 8, hipMemcpyDeviceToDevice,
                     stream) != hipSuccess)
    return ROM_EHIP;
  return ROM_OK;
}

}  // extern "C"
