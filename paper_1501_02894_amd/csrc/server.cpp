// Continuous-batching encode server.
//
// Requests (host images, each with its own thresholds and Technique-1 /
// identity-only flags over the server's block sizes) are queued by
// fe_server_submit.  A worker thread runs steps:
//   1. admission: queued requests enter in arrival order while a slot is
//      free and their device footprint fits: image, output, per-request
//      ordering scratch (byte arena) and their top tiles' record slots and
//      occupancy masks (tile arena).  The image is copied to the device on
//      one of two copy streams;
//   2. one launch of the fused MNS kernel over up to `step_blocks` blocks of
//      top tiles taken first-come first-served from every admitted request
//      whose image has arrived: mixed image sizes share the launch, and a
//      large image is spread over several steps; each block carries its
//      request's parameter set, so requests with different thresholds share
//      the launch too;
//   3. a request whose last block has run gets its stream ordered by a
//      kernel that writes the records and their count straight into the
//      request's pinned host buffer; the request completes when that
//      kernel's event has fired.
// The compute stream waits for a request's image copy on the device
// (stream-event wait), so the host never round-trips between stages.
// Records of a request live in its own tile slots, so they do not depend on
// what else shares the steps.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "fe.h"
#include "fe_common.h"
#include "fe_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) in units of `granule` (host-side
// bookkeeping of a device or pinned host allocation, or of tile slots).
class Arena {
 public:
  void reset(size_t size, size_t granule) {
    free_.clear();
    g_ = granule;
    size_ = size / g_ * g_;
    used_ = 0;
    if (size_) free_[0] = size_;
  }
  size_t round(size_t n) const { return (n + g_ - 1) / g_ * g_; }
  // offset, or SIZE_MAX when no free run is long enough
  size_t alloc(size_t n) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        used_ += n;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t n) {
    n = round(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, g_ = 1;
};

// Queued -> Copying (a large image's copy issued) -> Running (steps take its
// blocks; a small image's request goes there at once) -> Ordering (last
// block launched) -> Done / Failed.
enum class ReqState { Queued, Copying, Running, Ordering, Done, Failed };

struct Request {
  uint64_t id = 0;
  uint32_t w = 0, h = 0, pitch = 0;
  uint32_t tiles_x = 0, tiles_y = 0, groups_x = 0;
  uint64_t tiles = 0, blocks = 0, next_block = 0;
  uint32_t thr[4] = {0, 0, 0, 0};        // MSE thresholds of levels 1..L-1
  uint32_t flags = 0;                    // FE_PHASE2 / FE_IDENTITY_ONLY
  size_t cap = 0;                        // device output capacity (transforms)
  size_t chunks = 0;
  size_t hin_off = 0, hin_len = 0;       // pinned host input copy
  const uint8_t* hsrc = nullptr;         // or the caller's pinned image (zero-copy submit)
  uint32_t hstride = 0;                  // its row pitch
  size_t dev_off = 0, dev_len = 0;       // byte arena region
  size_t img_off = 0, csum_off = 0, cbase_off = 0;
  size_t tile_base = 0, tile_len = 0;    // tile arena range
  size_t hout_off = 0, hout_len = 0;     // pinned host output: records, then 2 x u64 offsets
  int slot = -1;                         // admission slot: owns ev_copied / ev_done of that slot
  int copy_stream = -1;                  // the copy stream of its image, while Copying
  size_t copy_bytes = 0;
  bool waited = false;                   // compute stream already waits on the copy event
  bool fetching = false;                 // fe_server_poll is copying the records out (lock not held)
  ReqState state = ReqState::Queued;
  size_t n_out = 0;
  // submitted, admitted (image copy issued), first and last step launched,
  // found complete
  Clock::time_point t_submit, t_admit, t_first, t_last, t_done;
  fe_status error = FE_OK;
};

}  // namespace

struct fe_server {
  int device = 0;
  fe_params params{};
  int L = 0, cells = 0;                  // fused levels; record cells per tile
  bool ext = false;                      // trees down to 2 x 2 (b_min = 2)
  uint4* fine_list = nullptr;            // ext: the step's 4 x 4 ranges that go on to 2 x 2
  uint32_t* fine_count = nullptr;
  uint64_t fine_cap = 0;
  fe::TileShape shape{};
  // image copies go to whichever of two streams has fewer bytes in flight
  // (back-to-back host-to-device copies of a request pool move about 47 GB/s
  // on one stream, 55 on two; a small image is not queued behind a large one
  // while the other stream is free)
  static constexpr int kCopyStreams = 2;
  hipStream_t compute = nullptr, copy[kCopyStreams] = {nullptr, nullptr};
  int next_copy = 0;                     // tie break between equally loaded streams
  size_t copy_pending[kCopyStreams] = {0, 0};   // bytes of Copying requests (worker thread only)
  static constexpr size_t kDirectCopyBytes = 1u << 20;   // up to this, a request need not wait for its copy
  uint8_t* dev_base = nullptr;           // byte arena memory
  uint4* staging = nullptr;              // tile arena: record slots
  uint64_t* masks = nullptr;             // tile arena: occupancy
  uint8_t* host_base = nullptr;          // pinned host arena
  Arena dev_arena, tile_arena, host_arena;
  std::vector<int> free_slots;
  uint32_t max_slots = 0, step_blocks = 0;
  fe::BlockDesc* h_desc[2] = {nullptr, nullptr};
  fe::BlockDesc* d_desc[2] = {nullptr, nullptr};
  std::vector<uint32_t> wg_words;        // a step's per-block parameter words (worker thread)
  hipEvent_t step_done[2] = {nullptr, nullptr};
  int step_slot = 0;
  std::vector<hipEvent_t> ev_copied, ev_done;   // per admission slot
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Request*> queued;
  std::deque<Request*> ordering;         // ordering kernels queued on the compute stream, in launch order
  std::deque<uint64_t> completions;      // finished ids not yet reported by fe_server_wait
  std::vector<Request*> active;          // admitted, not yet done
  std::map<uint64_t, Request*> all;      // by id, until fetched
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  uint64_t steps = 0, blocks_run = 0, completed = 0;
};

namespace {

size_t r256(size_t n) { return (n + 255) & ~(size_t)255; }

// Device byte footprint of a request (image and ordering scratch); its
// tile slots are accounted in the tile arena, its output in pinned host
// memory.
size_t byte_footprint(const Request* r) {
  return r256((size_t)r->pitch * r->h) + r256(r->chunks * 4) + r256((r->chunks + 1) * 8);
}

size_t host_out_bytes(const Request* r) { return r->cap * 16 + 16; }

// Bytes of a step's upload: `blocks` block descriptors, their parameter
// words, then `imgs` image entries.
size_t desc_bytes(uint32_t blocks, size_t imgs) {
  return (size_t)blocks * (sizeof(fe::BlockDesc) + fe::kWgParamWords * sizeof(uint32_t)) + imgs * sizeof(fe::ImgDev);
}

// Tile slots of a request: its workgroup blocks, each a full GX x GY group
// (record slots are laid out per block).
size_t slot_tiles(const fe_server* s, const Request* r) {
  return (size_t)r->blocks * (size_t)(s->shape.gx * s->shape.gy);
}

void release_request(fe_server* s, Request* r) {
  if (r->dev_len) s->dev_arena.release(r->dev_off, r->dev_len);
  if (r->tile_len) s->tile_arena.release(r->tile_base, r->tile_len);
  if (r->hin_len) s->host_arena.release(r->hin_off, r->hin_len);
  if (r->hout_len) s->host_arena.release(r->hout_off, r->hout_len);
  if (r->slot >= 0) s->free_slots.push_back(r->slot);
  r->dev_len = r->tile_len = r->hin_len = r->hout_len = 0;
  r->slot = -1;
}

// Release a fetched request and drop it from the completion queue.
void forget(fe_server* s, Request* r) {
  release_request(s, r);
  auto c = std::find(s->completions.begin(), s->completions.end(), r->id);
  if (c != s->completions.end()) s->completions.erase(c);
}

void fail_request(Request* r) {
  r->state = ReqState::Failed;
  r->error = FE_ERR_DEVICE;
}

// Admit queued requests in arrival order while slots and memory allow, and
// start their image copies.  Lock held on entry and exit; released while
// the copies are issued.
bool admit(fe_server* s, std::unique_lock<std::mutex>& lk) {
  std::vector<Request*> adm;
  while (!s->queued.empty() && !s->free_slots.empty()) {
    Request* r = s->queued.front();
    const size_t need = byte_footprint(r);
    const size_t off = s->dev_arena.alloc(need);
    if (off == SIZE_MAX) break;   // head of the queue waits for memory
    const size_t tlen = slot_tiles(s, r);
    const size_t tb = s->tile_arena.alloc(tlen);
    if (tb == SIZE_MAX) {
      s->dev_arena.release(off, need);
      break;
    }
    const size_t hout = s->host_arena.alloc(host_out_bytes(r));
    if (hout == SIZE_MAX) {
      s->tile_arena.release(tb, tlen);
      s->dev_arena.release(off, need);
      break;
    }
    s->queued.pop_front();
    r->t_admit = Clock::now();
    r->dev_off = off;
    r->dev_len = need;
    r->img_off = off;
    r->csum_off = r->img_off + r256((size_t)r->pitch * r->h);
    r->cbase_off = r->csum_off + r256(r->chunks * 4);
    r->hout_off = hout;
    r->hout_len = host_out_bytes(r);
    r->tile_base = tb;
    r->tile_len = tlen;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->active.push_back(r);       // still Queued: run_step skips it
    adm.push_back(r);
  }
  if (adm.empty()) return false;
  // only this thread touches admitted requests' device state
  lk.unlock();
  std::vector<char> ok(adm.size(), 0);
  for (size_t k = 0; k < adm.size(); ++k) {
    Request* r = adm[k];
    int ci = s->next_copy;
    for (int c = 0; c < fe_server::kCopyStreams; ++c)
      if (s->copy_pending[c] < s->copy_pending[ci]) ci = c;
    s->next_copy = (ci + 1) % fe_server::kCopyStreams;
    const hipStream_t cs = s->copy[ci];
    const size_t bytes = (size_t)r->pitch * r->h;
    // a small copy on a stream with no large one ahead of it is done within
    // tens of microseconds: its request joins the next step at once (the
    // step waits on the copy's event on the device); the others are polled
    const bool gated = bytes > fe_server::kDirectCopyBytes || s->copy_pending[ci] > 0;
    // the image (the encode kernel writes every tile's mask whole)
    // rows of equal pitch on both sides are one linear copy (a pitched copy
    // is slower even when it covers the same bytes)
    hipError_t e;
    if (!r->hsrc)
      e = hipMemcpyAsync(s->dev_base + r->img_off, s->host_base + r->hin_off, (size_t)r->pitch * r->h,
                         hipMemcpyHostToDevice, cs);
    else if (r->hstride == r->pitch)
      e = hipMemcpyAsync(s->dev_base + r->img_off, r->hsrc, (size_t)r->pitch * (r->h - 1) + r->w,
                         hipMemcpyHostToDevice, cs);
    else
      e = hipMemcpy2DAsync(s->dev_base + r->img_off, r->pitch, r->hsrc, r->hstride, r->w, r->h,
                           hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipEventRecord(s->ev_copied[r->slot], cs);
    ok[k] = e == hipSuccess;
    if (ok[k] && gated) {
      r->copy_stream = ci;
      r->copy_bytes = bytes;
      s->copy_pending[ci] += bytes;
    }
  }
  lk.lock();
  for (size_t k = 0; k < adm.size(); ++k) {
    if (ok[k]) adm[k]->state = adm[k]->copy_stream >= 0 ? ReqState::Copying : ReqState::Running;
    else fail_request(adm[k]);
  }
  return true;
}

// Requests whose polled image copy has completed become Running, so that no
// step waits on a large copy still in flight (a step holding a 16 Mpx
// image's first blocks would otherwise hold back every request in it for
// the copy's 0.3-0.7 ms).  Lock held.  Returns true on any change.
bool copied(fe_server* s) {
  bool any = false;
  for (Request* r : s->active) {
    if (r->state != ReqState::Copying) continue;
    const hipError_t q = hipEventQuery(s->ev_copied[r->slot]);
    if (q == hipErrorNotReady) continue;
    s->copy_pending[r->copy_stream] -= r->copy_bytes;
    r->copy_stream = -1;
    r->copy_bytes = 0;
    if (q == hipSuccess) r->state = ReqState::Running;
    else fail_request(r);
    any = true;
  }
  return any;
}

// One step: a single launch over up to step_blocks blocks.  Returns true if
// it launched work.  Lock held on entry and exit.
bool run_step(fe_server* s, std::unique_lock<std::mutex>& lk) {
  std::vector<Request*> ready;
  for (Request* r : s->active)
    if (r->state == ReqState::Running && r->next_block < r->blocks) ready.push_back(r);
  if (ready.empty()) return false;
  const int slot = s->step_slot;
  s->step_slot ^= 1;
  lk.unlock();
  (void)hipEventSynchronize(s->step_done[slot]);   // its descriptor buffer is free again
  lk.lock();
  fe::BlockDesc* hd = s->h_desc[slot];
  uint32_t n = 0;
  std::vector<Request*> finishing, first_time, in_step;
  // per-block parameter words, written beside the descriptors and moved
  // behind the last one before the upload
  std::vector<uint32_t>& hp = s->wg_words;
  hp.resize((size_t)s->step_blocks * fe::kWgParamWords);
  for (Request* r : ready) {
    if (n >= s->step_blocks) break;
    if (!r->waited) {
      first_time.push_back(r);
      r->waited = true;
      r->t_first = Clock::now();
    }
    in_step.push_back(r);
    while (r->next_block < r->blocks && n < s->step_blocks) {
      const uint64_t b = r->next_block++;
      const uint32_t gyi = (uint32_t)(b / r->groups_x), gxi = (uint32_t)(b - (uint64_t)gyi * r->groups_x);
      const uint32_t tx0 = gxi * (uint32_t)s->shape.gx, ty0 = gyi * (uint32_t)s->shape.gy;
      fe::BlockDesc& d = hd[n++];
      d.data = s->dev_base + r->img_off;
      d.tg0 = r->tile_base + (uint64_t)ty0 * r->tiles_x + tx0;
      d.stride = r->pitch;
      d.wh = (r->w - 1u) | ((r->h - 1u) << 16);
      d.t0 = tx0 | (ty0 << 16);
      d.sblk = (uint32_t)(r->tile_base / (size_t)(s->shape.gx * s->shape.gy) + b);
      uint32_t* w = hp.data() + (size_t)(n - 1) * fe::kWgParamWords;
      for (int l = 0; l < 4; ++l) w[l] = r->thr[l];
      w[4] = r->flags;
      w[5] = w[6] = w[7] = 0u;
    }
    if (r->next_block == r->blocks) {
      finishing.push_back(r);
      r->t_last = Clock::now();
    }
  }
  // one upload: the n descriptors, their parameter words, then the
  // finishing requests' image entries for their ordering kernels (blocks
  // numbered from 0 within the request's slot range)
  memcpy(hd + n, hp.data(), (size_t)n * fe::kWgParamWords * sizeof(uint32_t));
  fe::ImgDev* him = reinterpret_cast<fe::ImgDev*>(reinterpret_cast<uint32_t*>(hd + n) + (size_t)n * fe::kWgParamWords);
  for (size_t j = 0; j < finishing.size(); ++j) {
    const Request* r = finishing[j];
    fe::ImgDev& im = him[j];
    im = fe::ImgDev{};
    im.data = s->dev_base + r->img_off;
    im.width = r->w;
    im.height = r->h;
    im.stride = r->pitch;
    im.tiles_x = r->tiles_x;
    im.tiles_y = r->tiles_y;
    im.groups_x = r->groups_x;
    im.groups_y = (uint32_t)(r->blocks / r->groups_x);
  }
  // ext: the step's requests by tile-arena base, for the 2 x 2 level to
  // find each listed range's image
  fe::ImgDev* hx = him + finishing.size();
  if (s->ext) {
    std::sort(in_step.begin(), in_step.end(), [](const Request* x, const Request* y) { return x->tile_base < y->tile_base; });
    for (size_t j = 0; j < in_step.size(); ++j) {
      const Request* r = in_step[j];
      fe::ImgDev& im = hx[j];
      im = fe::ImgDev{};
      im.data = s->dev_base + r->img_off;
      im.width = r->w;
      im.height = r->h;
      im.stride = r->pitch;
      im.fine_flags = r->flags;
      im.fine_thr = r->thr[s->L - 1];
      im.tile_first = r->tile_base;
    }
  }
  const size_t n_x = s->ext ? in_step.size() : 0;
  const size_t upload = desc_bytes(n, finishing.size() + n_x);
  const uint32_t* dparams = reinterpret_cast<const uint32_t*>(s->d_desc[slot] + n);
  const fe::ImgDev* dim = reinterpret_cast<const fe::ImgDev*>(dparams + (size_t)n * fe::kWgParamWords);
  const fe::ImgDev* dx_tab = dim + finishing.size();
  lk.unlock();
  hipError_t e = hipSuccess;
  for (Request* r : first_time)
    if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, s->ev_copied[r->slot], 0);   // the image
  if (e == hipSuccess) e = hipMemcpyAsync(s->d_desc[slot], hd, upload, hipMemcpyHostToDevice, s->compute);
  if (e == hipSuccess) {
    fe::EncodeArgs a{};
    a.blocks = s->d_desc[slot];
    a.n_imgs = 1;
    a.n_wg = n;
    a.wg_params = dparams;
    a.staging = s->staging;
    a.masks = s->masks;
    if (!s->ext) {
      e = fe::launch_mns_tiles((int)s->params.b_max, s->L, s->shape, a, s->compute);
    } else {
      a.fine_list = s->fine_list;
      a.fine_count = s->fine_count;
      e = fe::launch_zero_u32(s->fine_count, 1, s->compute);
      if (e == hipSuccess) e = fe::launch_mns_tiles_ext((int)s->params.b_max, s->L, s->shape, a, s->compute);
      if (e == hipSuccess) {
        fe::FinishArgs f{};
        f.imgs = dx_tab;
        f.n_imgs = (uint32_t)n_x;
        f.list = s->fine_list;
        f.count = s->fine_count;
        f.level = (uint32_t)s->L;
        f.per_image = 1;
        f.nt = (uint32_t)(s->shape.gx * s->shape.gy);
        f.cells = (uint32_t)s->cells;
        f.staging = s->staging;
        f.masks = s->masks;
        const uint64_t bm4 = s->params.b_max / 4;
        e = fe::launch_fine_finish(f, (uint64_t)n * (uint64_t)(s->shape.gx * s->shape.gy) * bm4 * bm4, s->compute);
      }
    }
  }
  for (size_t j = 0; j < finishing.size(); ++j) {
    Request* r = finishing[j];
    if (e != hipSuccess) break;
    // records and offsets go straight to the pinned host output
    uint8_t* hout = s->host_base + r->hout_off;
    e = fe::launch_scatter(dim + j, 1, nullptr, r->tiles, s->cells, s->shape, s->masks + r->tile_base,
                           reinterpret_cast<uint32_t*>(s->dev_base + r->csum_off),
                           reinterpret_cast<uint64_t*>(s->dev_base + r->cbase_off),
                           s->staging + r->tile_base * (size_t)(s->cells + 1), reinterpret_cast<uint4*>(hout), r->cap,
                           reinterpret_cast<uint64_t*>(hout + r->cap * 16), s->compute);
    if (e == hipSuccess) e = hipEventRecord(s->ev_done[r->slot], s->compute);
  }
  if (e == hipSuccess) e = hipEventRecord(s->step_done[slot], s->compute);
  lk.lock();
  s->steps++;
  s->blocks_run += n;
  for (Request* r : finishing) {
    if (e != hipSuccess) {
      fail_request(r);
    } else {
      r->state = ReqState::Ordering;
      s->ordering.push_back(r);
    }
  }
  if (e != hipSuccess)
    for (Request* r : ready) fail_request(r);
  return true;
}

// Requests whose ordering kernel has finished complete.  Lock held.
// Returns true on any progress.
bool finish(fe_server* s) {
  bool any = false;
  // the ordering kernels run in launch order on the compute stream, so the
  // requests complete in that order: query from the oldest until one is
  // still running (one event query per completion, not per request)
  while (!s->ordering.empty()) {
    Request* r = s->ordering.front();
    if (r->state == ReqState::Ordering && hipEventQuery(s->ev_done[r->slot]) != hipSuccess) break;
    s->ordering.pop_front();
    if (r->state != ReqState::Ordering) continue;   // failed meanwhile
    uint64_t total = 0;
    memcpy(&total, s->host_base + r->hout_off + r->cap * 16 + 8, 8);
    r->n_out = (size_t)total;
    r->state = r->n_out <= r->cap ? ReqState::Done : ReqState::Failed;
    if (r->state == ReqState::Failed) r->error = FE_ERR_DEVICE;
    r->t_done = Clock::now();
    s->completed++;
    any = true;
  }
  for (size_t i = 0; i < s->active.size();) {
    Request* r = s->active[i];
    if (r->state == ReqState::Done || r->state == ReqState::Failed) {
      // the device side is no longer needed; the host output stays until fetched
      if (r->dev_len) s->dev_arena.release(r->dev_off, r->dev_len);
      if (r->tile_len) s->tile_arena.release(r->tile_base, r->tile_len);
      if (r->hin_len) s->host_arena.release(r->hin_off, r->hin_len);
      if (r->slot >= 0) s->free_slots.push_back(r->slot);
      r->dev_len = r->tile_len = r->hin_len = 0;
      r->slot = -1;
      s->active.erase(s->active.begin() + i);
      s->completions.push_back(r->id);
      any = true;
      continue;
    }
    ++i;
  }
  return any;
}

// The first host-to-device copy of a size class on a new stream has been
// measured at 7-11 ms (the runtime sets up that copy path on first use), once
// per server; a step that met it held back every request in flight.
// Creation takes them instead: sizes from 64 B up by factors of 4, for the
// descriptor upload on the compute stream and for image copies on the copy
// streams.  The copied bytes are placeholders that nothing reads.
bool warm_transfers(fe_server* s, size_t desc_max, size_t image_max) {
  hipError_t e = hipSuccess;
  for (size_t n = 64;; n *= 4) {
    if (n <= 4 * desc_max)
      e = hipMemcpyAsync(s->d_desc[0], s->h_desc[0], std::min(n, desc_max), hipMemcpyHostToDevice, s->compute);
    for (int c = 0; e == hipSuccess && c < fe_server::kCopyStreams; ++c)
      e = hipMemcpyAsync(s->dev_base, s->host_base, std::min(n, image_max), hipMemcpyHostToDevice, s->copy[c]);
    if (e != hipSuccess || (n >= desc_max && n >= image_max)) break;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->compute);
  for (int c = 0; e == hipSuccess && c < fe_server::kCopyStreams; ++c) e = hipStreamSynchronize(s->copy[c]);
  return e == hipSuccess;
}

void worker_main(fe_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool progress = admit(s, lk);
    progress |= copied(s);
    progress |= run_step(s, lk);
    const size_t before = s->completions.size();
    progress |= finish(s);
    if (s->completions.size() != before) s->done_cv.notify_all();
    if (progress) continue;
    if (s->active.empty()) {
      s->cv.wait_for(lk, std::chrono::microseconds(500));
    } else {
      // work is on the device: poll its events without sleeping
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

fe_status fe_server_create(int device, const fe_params* p, size_t hbm_budget, size_t host_budget,
                           uint32_t max_slots, uint32_t step_blocks, fe_server** out) {
  fe::clear_error();
  if (!out || hbm_budget < (8u << 20) || host_budget < (1u << 20) || max_slots == 0 || step_blocks == 0)
    return fe::fail(FE_ERR_INVALID, "bad server arguments");
  *out = nullptr;
  fe_status st = fe::check_params(p);
  if (st != FE_OK) return st;
  if (p->flags & (FE_FULL_SEARCH | FE_LOCAL_SEARCH)) return fe::fail(FE_ERR_INVALID, "the server runs MNS only");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fe::fail(FE_ERR_DEVICE, "no HIP device %d", device);
  fe_server* s = new fe_server();
  s->device = device;
  s->params = *p;
  // b_min = 2: the fused kernel's EXT form down to 4 x 4 (default shape),
  // then the 2 x 2 level; record cells are 2 x 2 units
  s->ext = p->b_min < 4;
  s->L = fe::levels_of(p->b_max, s->ext ? 4u : p->b_min);
  s->cells = 1 << (2 * (s->L - 1 + (s->ext ? 1 : 0)));
  fe::TileShape shapes[16];
  if (fe::encode_shapes((int)p->b_max, s->L, shapes, 16) == 0) {
    delete s;
    return fe::fail(FE_ERR_INVALID, "no kernel for these block sizes");
  }
  s->shape = shapes[0];
  s->max_slots = max_slots;
  s->step_blocks = step_blocks;
  // a quarter of the budget holds tile slots (records + masks), the rest
  // images, outputs and ordering scratch
  const size_t tile_bytes = (size_t)(s->cells + 1) * 16 + 8;   // record slots and mask
  size_t tiles_cap = (hbm_budget / 4) / tile_bytes;
  // the 2 x 2 level's list holds 32-bit record slots
  if (s->ext) tiles_cap = std::min<size_t>(tiles_cap, ((1ull << 32) - 1) / (size_t)(s->cells + 1));
  const size_t byte_budget = hbm_budget - tiles_cap * tile_bytes;
  (void)hipSetDevice(device);
  bool ok = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->copy[0], hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->copy[1], hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&s->dev_base), byte_budget) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&s->staging), tiles_cap * (s->cells + 1) * 16) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&s->masks), tiles_cap * 8) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&s->host_base), host_budget, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ok && k < 2; ++k)
    // per step: the block descriptors and their parameter words, then one
    // image entry per finishing request and (ext) one per request of the step
    ok = hipHostMalloc(reinterpret_cast<void**>(&s->h_desc[k]), desc_bytes(step_blocks, 2 * (size_t)step_blocks),
                       hipHostMallocDefault) == hipSuccess &&
         hipMalloc(reinterpret_cast<void**>(&s->d_desc[k]), desc_bytes(step_blocks, 2 * (size_t)step_blocks)) ==
             hipSuccess &&
         hipEventCreateWithFlags(&s->step_done[k], hipEventDisableTiming) == hipSuccess;
  if (ok && s->ext) {
    const uint64_t bm4 = p->b_max / 4;
    s->fine_cap = (uint64_t)step_blocks * (uint64_t)(s->shape.gx * s->shape.gy) * bm4 * bm4;
    ok = hipMalloc(reinterpret_cast<void**>(&s->fine_list), std::max<uint64_t>(s->fine_cap, 1) * 16) == hipSuccess &&
         hipMalloc(reinterpret_cast<void**>(&s->fine_count), 4) == hipSuccess;
  }
  s->ev_copied.assign(max_slots, nullptr);
  s->ev_done.assign(max_slots, nullptr);
  for (uint32_t k = 0; ok && k < max_slots; ++k)
    ok = hipEventCreateWithFlags(&s->ev_copied[k], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&s->ev_done[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    fe_server_destroy(s);
    return fe::fail(FE_ERR_OOM, "server allocation failed");
  }
  if (!warm_transfers(s, desc_bytes(step_blocks, 2 * (size_t)step_blocks),
                      std::min<size_t>({byte_budget, host_budget, (size_t)64 << 20}))) {
    fe_server_destroy(s);
    return fe::fail(FE_ERR_DEVICE, "server stream set-up failed");
  }
  s->dev_arena.reset(byte_budget, 256);
  // tile slots are handed out in whole blocks of the tile shape
  s->tile_arena.reset(tiles_cap, (size_t)(s->shape.gx * s->shape.gy));
  s->host_arena.reset(host_budget, 256);
  for (int k = (int)max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return FE_OK;
}

void fe_server_destroy(fe_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  if (s->compute) (void)hipStreamSynchronize(s->compute);
  for (hipStream_t c : s->copy)
    if (c) (void)hipStreamSynchronize(c);
  for (auto& kv : s->all) {
    release_request(s, kv.second);
    delete kv.second;
  }
  for (int k = 0; k < 2; ++k) {
    if (s->h_desc[k]) (void)hipHostFree(s->h_desc[k]);
    if (s->d_desc[k]) (void)hipFree(s->d_desc[k]);
    if (s->step_done[k]) (void)hipEventDestroy(s->step_done[k]);
  }
  for (hipEvent_t ev : s->ev_copied)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : s->ev_done)
    if (ev) (void)hipEventDestroy(ev);
  if (s->dev_base) (void)hipFree(s->dev_base);
  if (s->staging) (void)hipFree(s->staging);
  if (s->fine_list) (void)hipFree(s->fine_list);
  if (s->fine_count) (void)hipFree(s->fine_count);
  if (s->masks) (void)hipFree(s->masks);
  if (s->host_base) (void)hipHostFree(s->host_base);
  if (s->compute) (void)hipStreamDestroy(s->compute);
  for (hipStream_t c : s->copy)
    if (c) (void)hipStreamDestroy(c);
  delete s;
}

namespace {

// A new request for a W x H image (not yet queued), or NULL with the error
// set.  p: its parameters (NULL: the server's), which may differ from the
// server's in their thresholds and FE_PHASE2 / FE_IDENTITY_ONLY flags only.
Request* new_request(fe_server* s, uint32_t w, uint32_t h, uint32_t stride, const fe_params* p, fe_status& st) {
  if (!p) p = &s->params;
  st = fe::check_params(p);
  if (st != FE_OK) return nullptr;
  if (p->b_max != s->params.b_max || p->b_min != s->params.b_min ||
      (p->flags & ~(uint32_t)(FE_PHASE2 | FE_IDENTITY_ONLY)) != 0) {
    st = fe::fail(FE_ERR_INVALID, "request parameters must keep the server's b_max / b_min and run MNS or no-search");
    return nullptr;
  }
  st = fe::check_shape(w, h, stride, s->params.b_max);
  if (st != FE_OK) return nullptr;
  Request* r = new Request();
  for (int l = 0; l < 4; ++l) r->thr[l] = l < (int)p->n_thr ? p->mse_thr[l] : 0u;
  r->flags = p->flags;
  r->w = w;
  r->h = h;
  r->pitch = w;   // W is a multiple of b_max >= 4
  r->tiles_x = w / s->params.b_max;
  r->tiles_y = h / s->params.b_max;
  r->groups_x = (r->tiles_x + s->shape.gx - 1) / s->shape.gx;
  r->tiles = (uint64_t)r->tiles_x * r->tiles_y;
  r->blocks = (uint64_t)r->groups_x * ((r->tiles_y + s->shape.gy - 1) / s->shape.gy);
  r->cap = fe_max_transforms(w, h, s->params.b_min);
  r->chunks = (size_t)((r->tiles + fe::kChunkTiles - 1) / fe::kChunkTiles);
  if (byte_footprint(r) > s->dev_arena.size() || slot_tiles(s, r) > s->tile_arena.size()) {
    delete r;
    st = fe::fail(FE_ERR_OOM, "request is larger than the server's device budget");
    return nullptr;
  }
  return r;
}

// Queue a prepared request (lock not held on entry).
void enqueue(fe_server* s, Request* r, uint64_t* req) {
  std::unique_lock<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  s->queued.push_back(r);
  s->all[r->id] = r;
  *req = r->id;
  lk.unlock();
  s->cv.notify_all();
}

}  // namespace

fe_status fe_server_submit(fe_server* s, const uint8_t* h_img, uint32_t w, uint32_t h, uint32_t stride,
                           const fe_params* params, uint64_t* req) {
  fe::clear_error();
  if (!s || !h_img || !req) return fe::fail(FE_ERR_INVALID, "NULL argument");
  fe_status st;
  Request* r = new_request(s, w, h, stride, params, st);
  if (!r) return st;
  std::unique_lock<std::mutex> lk(s->mu);
  const size_t hin = s->host_arena.alloc((size_t)r->pitch * h);
  if (hin == SIZE_MAX) {
    delete r;
    return fe::fail(FE_ERR_BUSY, "host staging is full");
  }
  r->hin_off = hin;
  r->hin_len = (size_t)r->pitch * h;
  r->t_submit = Clock::now();
  lk.unlock();
  // the staging region is reserved: copy into it without holding the lock
  uint8_t* dst = s->host_base + hin;
  if (stride == r->pitch) {
    memcpy(dst, h_img, (size_t)r->pitch * h);
  } else {
    for (uint32_t y = 0; y < h; ++y) memcpy(dst + (size_t)y * r->pitch, h_img + (size_t)y * stride, w);
  }
  enqueue(s, r, req);
  return FE_OK;
}

fe_status fe_server_submit_pinned(fe_server* s, const uint8_t* h_img, uint32_t w, uint32_t h, uint32_t stride,
                                  const fe_params* params, uint64_t* req) {
  fe::clear_error();
  if (!s || !h_img || !req) return fe::fail(FE_ERR_INVALID, "NULL argument");
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, h_img) != hipSuccess || attr.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fe::fail(FE_ERR_INVALID, "image is not in pinned host memory");
  }
  fe_status st;
  Request* r = new_request(s, w, h, stride, params, st);
  if (!r) return st;
  r->hsrc = h_img;
  r->hstride = stride;
  r->t_submit = Clock::now();
  enqueue(s, r, req);
  return FE_OK;
}

fe_status fe_server_poll(fe_server* s, uint64_t req, fe_transform* h_out, size_t cap, size_t* n, int* done,
                         double* latency_ms) {
  fe::clear_error();
  if (!s || !done) return fe::fail(FE_ERR_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(req);
  if (it == s->all.end()) return fe::fail(FE_ERR_INVALID, "unknown request %llu", (unsigned long long)req);
  Request* r = it->second;
  if (r->fetching) return fe::fail(FE_ERR_BUSY, "request %llu is being fetched by another call", (unsigned long long)req);
  if (r->state == ReqState::Failed) {
    const fe_status e = r->error;
    if (std::find(s->active.begin(), s->active.end(), r) == s->active.end()) {
      forget(s, r);
      s->all.erase(it);
      delete r;
    }
    return fe::fail(e, "request failed on the device");
  }
  if (r->state != ReqState::Done) {
    *done = 0;
    return FE_OK;
  }
  *done = 1;
  if (n) *n = r->n_out;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (h_out) {
    if (cap < r->n_out) return fe::fail(FE_ERR_CAPACITY, "output holds %zu transforms, %zu needed", cap, r->n_out);
    // copy without the lock (the worker keeps stepping meanwhile); the
    // request's pinned output stays reserved until it is forgotten below
    r->fetching = true;
    const uint8_t* src = s->host_base + r->hout_off;
    const size_t bytes = r->n_out * sizeof(fe_transform);
    lk.unlock();
    memcpy(h_out, src, bytes);
    lk.lock();
    forget(s, r);
    s->all.erase(req);
    delete r;
  }
  return FE_OK;
}

fe_status fe_server_result(fe_server* s, uint64_t req, const fe_transform** recs, size_t* n, double* latency_ms) {
  fe::clear_error();
  if (!s || !recs || !n) return fe::fail(FE_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(req);
  if (it == s->all.end()) return fe::fail(FE_ERR_INVALID, "unknown request %llu", (unsigned long long)req);
  Request* r = it->second;
  if (r->fetching) return fe::fail(FE_ERR_BUSY, "request %llu is being fetched by another call", (unsigned long long)req);
  if (r->state == ReqState::Failed) {
    const fe_status e = r->error;
    if (std::find(s->active.begin(), s->active.end(), r) == s->active.end()) {
      forget(s, r);
      s->all.erase(it);
      delete r;
    }
    return fe::fail(e, "request failed on the device");
  }
  if (r->state != ReqState::Done) return fe::fail(FE_ERR_BUSY, "request %llu is not done", (unsigned long long)req);
  *recs = reinterpret_cast<const fe_transform*>(s->host_base + r->hout_off);
  *n = r->n_out;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  return FE_OK;
}

fe_status fe_server_release(fe_server* s, uint64_t req) {
  fe::clear_error();
  if (!s) return fe::fail(FE_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(req);
  if (it == s->all.end()) return fe::fail(FE_ERR_INVALID, "unknown request %llu", (unsigned long long)req);
  Request* r = it->second;
  if (r->fetching) return fe::fail(FE_ERR_BUSY, "request %llu is being fetched by another call", (unsigned long long)req);
  if (r->state != ReqState::Done && r->state != ReqState::Failed)
    return fe::fail(FE_ERR_BUSY, "request %llu is not finished", (unsigned long long)req);
  if (std::find(s->active.begin(), s->active.end(), r) != s->active.end())
    return fe::fail(FE_ERR_BUSY, "request %llu is still being retired", (unsigned long long)req);
  forget(s, r);
  s->all.erase(it);
  delete r;
  return FE_OK;
}

fe_status fe_server_request_times(fe_server* s, uint64_t req, double* ms, uint32_t n) {
  fe::clear_error();
  if (!s || (n && !ms)) return fe::fail(FE_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(req);
  if (it == s->all.end()) return fe::fail(FE_ERR_INVALID, "unknown request %llu", (unsigned long long)req);
  const Request* r = it->second;
  if (r->state != ReqState::Done) return fe::fail(FE_ERR_BUSY, "request %llu is not done", (unsigned long long)req);
  const Clock::time_point t[4] = {r->t_admit, r->t_first, r->t_last, r->t_done};
  for (uint32_t k = 0; k < n && k < 4; ++k)
    ms[k] = std::chrono::duration<double, std::milli>(t[k] - r->t_submit).count();
  return FE_OK;
}

fe_status fe_server_wait(fe_server* s, uint32_t timeout_us, uint64_t* req) {
  fe::clear_error();
  if (!s || !req) return fe::fail(FE_ERR_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), [s] { return !s->completions.empty(); }))
    return fe::fail(FE_ERR_BUSY, "no request finished within %u us", timeout_us);
  *req = s->completions.front();
  s->completions.pop_front();
  return FE_OK;
}

fe_status fe_server_stats(fe_server* s, uint64_t* steps, uint64_t* blocks, uint64_t* completed, size_t* hbm_used,
                          uint32_t* in_flight, uint32_t* queued) {
  fe::clear_error();
  if (!s) return fe::fail(FE_ERR_INVALID, "NULL server");
  std::lock_guard<std::mutex> g(s->mu);
  if (steps) *steps = s->steps;
  if (blocks) *blocks = s->blocks_run;
  if (completed) *completed = s->completed;
  if (hbm_used) *hbm_used = s->dev_arena.used() + s->tile_arena.used() * ((size_t)(s->cells + 1) * 16 + 8);
  if (in_flight) *in_flight = (uint32_t)s->active.size();
  if (queued) *queued = (uint32_t)s->queued.size();
  return FE_OK;
}

}  // extern "C"
