// pipeline.hip -- the streaming form: raw events in host memory in,
// compact tracks and primary vertices in host memory out, with several
// host-thread / HIP-stream pairs in flight (paper Sec. 2.2: raw data are
// copied to the GPU and only the objects the selections need come back;
// Sec. 3.2: every CPU thread drives one GPU stream so that transfers overlap
// with the kernels of the other streams).
//
// velo_pipeline_run first applies the global event cut on the host (events
// with more raw words than the cut are not processed, Sec. 2.3: the busiest
// events are removed before the sequence), splits the remaining events into
// batches, and hands batch k to slot k mod S.  A slot owns a stream, pinned
// staging buffers and device buffers sized for one batch; for every batch it
//   packs the batch's words and offsets into its pinned staging buffer,
//   copies them to the device (asynchronous, on its stream),
//   runs clustering, track finding, the fit (or the fit with the classifier)
//   and vertex finding,
//   gathers the tracks of the batch into dense 32-byte rows (k_track_rows,
//   after a scan of the per-event track counts, k_track_first),
//   copies the per-event counts and statuses and the vertices back, and
//   after a synchronisation of its own stream, exactly the rows that exist;
// then appends the rows to the caller's table.  The slots run concurrently,
// so one slot's copies overlap with the other slots' kernels.
#include <atomic>
#include <string.h>
#include <thread>
#include <vector>

namespace velo {

constexpr int kRowThreads = 256;

// first[e] = sum of the (clamped) track counts of events before e; first[E] = total
__global__ __launch_bounds__(1024) void k_track_first(const uint64_t* __restrict__ offsets,
                                                      uint32_t n_events, uint64_t n_pixels,
                                                      const uint32_t* __restrict__ n_tracks,
                                                      uint32_t* __restrict__ first) {
  __shared__ uint32_t tmp[2][1024 / kWave];
  uint32_t carry = 0;
  int buf = 0;
  for (uint32_t e0 = 0; e0 < n_events; e0 += 1024, buf ^= 1) {
    const uint32_t e = e0 + threadIdx.x;
    uint32_t c = 0;
    if (e < n_events) {
      const uint64_t b = offsets[e], end = offsets[e + 1];
      c = (b <= end && end <= n_pixels) ? event_tracks(n_tracks[e], (uint32_t)(end - b)) : 0u;
    }
    uint32_t tot;
    const uint32_t x = block_scan1<1024>(c, tmp[buf], &tot);
    if (e < n_events) first[e] = carry + x;
    carry += tot;
  }
  if (threadIdx.x == 0) first[n_events] = carry;
}

// dense rows of every event's tracks, at first[e] + t
__global__ __launch_bounds__(kRowThreads) void k_track_rows(const uint64_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ first,
                                                            const uint8_t* __restrict__ nhits,
                                                            velo_states s,
                                                            velo_track_row* __restrict__ rows) {
  const uint32_t e = blockIdx.x;
  const uint64_t base = offsets[e] / 3;
  const uint32_t f = first[e], n = first[e + 1] - f;
  for (uint32_t t = threadIdx.x; t < n; t += kRowThreads) {
    const uint64_t slot = base + t;
    velo_track_row r;
    r.x = s.x[slot];
    r.y = s.y[slot];
    r.z = s.z[slot];
    r.tx = s.tx[slot];
    r.ty = s.ty[slot];
    r.chi2 = s.chi2[slot];
    r.ndof = s.ndof[slot];
    r.accepted = s.accepted[slot];
    r.nhits = nhits[slot];
    r.pad = 0;
    rows[f + t] = r;
  }
}

// status of every event: clustering, track finding and vertex finding bits
__global__ void k_event_status(uint32_t n_events, const uint32_t* __restrict__ hs,
                               const uint32_t* __restrict__ ts, const uint32_t* __restrict__ ps,
                               uint32_t* __restrict__ out) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_events) out[e] = hs[e] | ts[e] | ps[e];
}

}  // namespace velo

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
}

struct Slot {
  hipStream_t stream = nullptr;
  // pinned staging
  uint32_t* h_px = nullptr;
  uint64_t* h_off = nullptr;
  uint32_t* h_first = nullptr;
  uint32_t* h_status = nullptr;
  uint32_t* h_npv = nullptr;
  float* h_pvz = nullptr;
  float* h_pvvar = nullptr;
  velo_track_row* h_rows = nullptr;
  // device
  uint32_t* d_px = nullptr;
  uint64_t* d_off = nullptr;
  velo_hits hits{};
  velo_tracks tracks{};
  velo_states states{};
  velo_pvs pvs{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* d_first = nullptr;
  uint32_t* d_status = nullptr;
  velo_track_row* d_rows = nullptr;
};

}  // namespace

struct velo_pipeline {
  velo_pipeline_config cfg{};
  velo_geometry geom{};
  velo_params params{};
  velo_pv_params pvp{};
  bool has_mlp = false;
  velo_mlp mlp{};
  int device = 0;
  std::vector<Slot> slots;
};

namespace {

void free_slot(Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  void* hp[] = {s.h_px, s.h_off, s.h_first, s.h_status, s.h_npv, s.h_pvz, s.h_pvvar, s.h_rows};
  for (void* p : hp)
    if (p) (void)hipHostFree(p);
  void* dp[] = {s.d_px, s.d_off, s.hits.x, s.hits.y, s.hits.key, s.hits.aux, s.hits.layer_start,
                s.hits.layer_nhits, s.hits.n_hits, s.hits.status, s.tracks.n_tracks, s.tracks.nhits,
                s.tracks.hit_idx, s.tracks.status, s.states.x, s.states.y, s.states.z, s.states.tx,
                s.states.ty, s.states.cov_x, s.states.cov_y, s.states.chi2, s.states.ndof,
                s.states.accepted, s.states.score, s.pvs.n_pv, s.pvs.z, s.pvs.var, s.pvs.weight,
                s.pvs.status, s.ws, s.d_first, s.d_status, s.d_rows};
  for (void* p : dp)
    if (p) (void)hipFree(p);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

hipError_t make_slot(Slot& s, uint32_t E, uint64_t N) {
  hipError_t e;
  const uint64_t cap = N / 3 > 0 ? N / 3 : 1;
  const size_t P = (size_t)E * VELO_MAX_PVS;
#define VELO_TRY(x) \
  if ((e = (x)) != hipSuccess) return e
  VELO_TRY(hipStreamCreate(&s.stream));
  VELO_TRY(hipHostMalloc((void**)&s.h_px, (N ? N : 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_off, (E + 1) * 8, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_first, (E + 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_status, (E ? E : 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_npv, (E ? E : 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_pvz, (P ? P : 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_pvvar, (P ? P : 1) * 4, hipHostMallocDefault));
  VELO_TRY(hipHostMalloc((void**)&s.h_rows, cap * sizeof(velo_track_row), hipHostMallocDefault));
  VELO_TRY(dalloc(&s.d_px, N));
  VELO_TRY(dalloc(&s.d_off, E + 1));
  VELO_TRY(dalloc(&s.hits.x, N));
  VELO_TRY(dalloc(&s.hits.y, N));
  VELO_TRY(dalloc(&s.hits.key, N));
  VELO_TRY(dalloc(&s.hits.aux, N));
  VELO_TRY(dalloc(&s.hits.layer_start, 27ull * E));
  VELO_TRY(dalloc(&s.hits.layer_nhits, 26ull * E));
  VELO_TRY(dalloc(&s.hits.n_hits, E));
  VELO_TRY(dalloc(&s.hits.status, E));
  VELO_TRY(dalloc(&s.tracks.n_tracks, E));
  VELO_TRY(dalloc(&s.tracks.nhits, cap));
  VELO_TRY(dalloc(&s.tracks.hit_idx, 26 * cap));
  VELO_TRY(dalloc(&s.tracks.status, E));
  VELO_TRY(dalloc(&s.states.x, cap));
  VELO_TRY(dalloc(&s.states.y, cap));
  VELO_TRY(dalloc(&s.states.z, cap));
  VELO_TRY(dalloc(&s.states.tx, cap));
  VELO_TRY(dalloc(&s.states.ty, cap));
  VELO_TRY(dalloc(&s.states.cov_x, 3 * cap));
  VELO_TRY(dalloc(&s.states.cov_y, 3 * cap));
  VELO_TRY(dalloc(&s.states.chi2, cap));
  VELO_TRY(dalloc(&s.states.ndof, cap));
  VELO_TRY(dalloc(&s.states.accepted, cap));
  VELO_TRY(dalloc(&s.states.score, cap));
  VELO_TRY(dalloc(&s.pvs.n_pv, E));
  VELO_TRY(dalloc(&s.pvs.z, P));
  VELO_TRY(dalloc(&s.pvs.var, P));
  VELO_TRY(dalloc(&s.pvs.weight, P));
  VELO_TRY(dalloc(&s.pvs.status, E));
  s.ws_bytes = velo_workspace_bytes(N, E);
  VELO_TRY(hipMalloc(&s.ws, s.ws_bytes));
  VELO_TRY(dalloc(&s.d_first, E + 1));
  VELO_TRY(dalloc(&s.d_status, E));
  VELO_TRY(dalloc(&s.d_rows, cap));
#undef VELO_TRY
  return hipSuccess;
}

struct Batch {
  uint64_t first_sel;  // index into the selected-event list
  uint32_t n;          // events
  uint64_t words;
};

struct RunShared {
  const uint32_t* px;
  const uint64_t* off;
  const std::vector<uint32_t>* sel;
  const std::vector<Batch>* batches;
  const velo_pipeline_result* out;
  std::atomic<uint64_t> rows{0};
  std::atomic<int> err{0};  // first velo_status error
};

velo_status slot_run(velo_pipeline* p, int k, RunShared* R) {
  Slot& s = p->slots[k];
  if (hipSetDevice(p->device) != hipSuccess) return VELO_ERR_HIP;
  const int S = (int)p->slots.size();
  const std::vector<uint32_t>& sel = *R->sel;
  const velo_pipeline_result* out = R->out;
  for (size_t bi = (size_t)k; bi < R->batches->size(); bi += (size_t)S) {
    if (R->err.load() != 0) return VELO_OK;
    const Batch& B = (*R->batches)[bi];
    // pack the batch into the pinned staging buffer
    uint64_t w = 0;
    for (uint32_t i = 0; i < B.n; ++i) {
      const uint32_t ev = sel[B.first_sel + i];
      const uint64_t a = R->off[ev], n = R->off[ev + 1] - a;
      s.h_off[i] = w;
      memcpy(s.h_px + w, R->px + a, n * 4);
      w += n;
    }
    s.h_off[B.n] = w;
    hipError_t e = hipMemcpyAsync(s.d_px, s.h_px, w * 4, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s.d_off, s.h_off, (B.n + 1) * 8, hipMemcpyHostToDevice, s.stream);
    if (e != hipSuccess) return VELO_ERR_HIP;
    velo_status st =
        p->has_mlp ? velo_reconstruct_mlp(s.d_px, s.d_off, B.n, w, &p->geom, &p->params, &p->mlp,
                                          &s.hits, &s.tracks, &s.states, s.ws, s.ws_bytes, s.stream)
                   : velo_reconstruct(s.d_px, s.d_off, B.n, w, &p->geom, &p->params, &s.hits,
                                      &s.tracks, &s.states, s.ws, s.ws_bytes, s.stream);
    if (st != VELO_OK) return st;
    st = velo_find_pvs(&s.tracks, &s.states, s.d_off, B.n, w, &p->pvp, &s.pvs, s.stream);
    if (st != VELO_OK) return st;
    hipLaunchKernelGGL(velo::k_track_first, dim3(1), dim3(1024), 0, s.stream, s.d_off, B.n, w,
                       s.tracks.n_tracks, s.d_first);
    hipLaunchKernelGGL(velo::k_track_rows, dim3(B.n), dim3(velo::kRowThreads), 0, s.stream, s.d_off,
                       s.d_first, s.tracks.nhits, s.states, s.d_rows);
    hipLaunchKernelGGL(velo::k_event_status, dim3((B.n + 255) / 256), dim3(256), 0, s.stream, B.n,
                       s.hits.status, s.tracks.status, s.pvs.status, s.d_status);
    e = hipGetLastError();
    const size_t P = (size_t)B.n * VELO_MAX_PVS;
    if (e == hipSuccess)
      e = hipMemcpyAsync(s.h_first, s.d_first, (B.n + 1) * 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s.h_status, s.d_status, B.n * 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s.h_npv, s.pvs.n_pv, B.n * 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_pvz, s.pvs.z, P * 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s.h_pvvar, s.pvs.var, P * 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return VELO_ERR_HIP;
    // exactly the rows that exist
    const uint32_t total = s.h_first[B.n];
    if (total) {
      e = hipMemcpyAsync(s.h_rows, s.d_rows, (size_t)total * sizeof(velo_track_row),
                         hipMemcpyDeviceToHost, s.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
      if (e != hipSuccess) return VELO_ERR_HIP;
    }
    const uint64_t r0 = R->rows.fetch_add(total);
    if (r0 + total > out->track_capacity) return VELO_ERR_WORKSPACE;
    memcpy(out->tracks + r0, s.h_rows, (size_t)total * sizeof(velo_track_row));
    for (uint32_t i = 0; i < B.n; ++i) {
      const uint32_t ev = sel[B.first_sel + i];
      out->status[ev] = s.h_status[i];
      out->n_tracks[ev] = s.h_first[i + 1] - s.h_first[i];
      out->first_track[ev] = r0 + s.h_first[i];
      if (out->n_pv) {
        out->n_pv[ev] = s.h_npv[i];
        memcpy(out->pv_z + (size_t)ev * VELO_MAX_PVS, s.h_pvz + (size_t)i * VELO_MAX_PVS,
               VELO_MAX_PVS * 4);
        memcpy(out->pv_var + (size_t)ev * VELO_MAX_PVS, s.h_pvvar + (size_t)i * VELO_MAX_PVS,
               VELO_MAX_PVS * 4);
      }
    }
  }
  return VELO_OK;
}

}  // namespace
