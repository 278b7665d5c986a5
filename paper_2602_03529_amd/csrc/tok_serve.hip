// Streaming request loop for the tokenizer: continuous batching of clips under
// an HBM budget (see the tok_server_* contract in include/tok.h).
//
// One device arena is allocated at create; requests draw their workspace,
// pixels, latents and reconstruction from it, so the request path never calls
// hipMalloc.  A scheduler thread polls completion events, returns memory and
// stream slots, and admits queued clips oldest-first, batching queued clips of
// identical shape into one launch.  Each clip's drop mask is applied on its own
// latent sub-range, so batching never changes a clip's result.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tok.h"

namespace {

using Clock = std::chrono::steady_clock;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over one device buffer; blocks coalesce on free.
class Arena {
 public:
  void init(char* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  char* alloc(size_t n) {
    n = align256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used_ += n;
        if (used_ > peak_) peak_ = used_;
        sizes_[off] = n;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p) {
    if (!p) return;
    const size_t off = (size_t)(p - base_);
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    const size_t n = s->second;
    sizes_.erase(s);
    used_ -= n;
    size_t start = off, end = off + n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == end) {  // merge with the following free block
      end += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the preceding free block
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        free_.erase(prev);
      }
    }
    free_[start] = end - start;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
  std::unordered_map<size_t, size_t> sizes_;
};

struct Shape {
  int T, H, W, T2, H2, W2;
  size_t pix, tok, xhat;  // elements per clip: pixels (bytes), latent tokens, reconstruction floats
  bool operator==(const Shape& o) const { return T == o.T && H == o.H && W == o.W; }
};

bool make_shape(int T, int H, int W, Shape* s) {
  if (T < 1 || (T - 1) % 4 || H < 4 || W < 4 || H % 4 || W % 4) return false;
  s->T = T; s->H = H; s->W = W;
  s->T2 = (T - 1) / 4 + 1; s->H2 = H / 4; s->W2 = W / 4;
  s->pix = (size_t)T * H * W * 3;
  s->tok = (size_t)s->T2 * s->H2 * s->W2;
  s->xhat = (size_t)T * H * W * 3;
  return true;
}

// Device bytes of the per-clip result block: codes, idx, keep, xhat.
size_t result_bytes(const Shape& s) {
  return align256(s.tok * 6 * 4) + align256(s.tok * 4) + align256(s.tok) + align256(s.xhat * 4);
}

struct Batch;

struct Request {
  uint64_t ticket;
  tok_request req;
  Shape shape;
  enum State { QUEUED, RUNNING, DONE, RELEASED } state = QUEUED;
  tok_status status = TOK_OK;
  Clock::time_point t_submit, t_admit, t_done;
  int batch_size = 0;
  char* results = nullptr;  // per-clip result block in the arena
};

struct Batch {
  std::vector<Request*> reqs;
  int slot = -1;
  char* scratch = nullptr;  // workspace + pixels, freed at completion
};

}  // namespace

struct tok_server {
  tok_model* model = nullptr;
  int device = 0;
  int max_batch = 1;
  char* mem = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<Batch*> slot_batch;  // nullptr = free slot
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  int finished = 0;
  bool stop = false;
  std::thread worker;

  // Workspace for a launch of n clips: whole-clip processing when it takes at
  // most a quarter of the arena, else causal temporal chunks (smaller, and
  // independent of the clip length).
  size_t ws_bytes(int n, const Shape& s) const {
    size_t whole = 0, stream = 0;
    tok_workspace_size(model, n, s.T, s.H, s.W, TOK_WS_ROUNDTRIP, &whole);
    if (whole * 4 <= arena.size()) return whole;
    tok_workspace_size(model, n, s.T, s.H, s.W, TOK_WS_ROUNDTRIP | TOK_WS_STREAM, &stream);
    return stream;
  }
  size_t scratch_bytes(int n, const Shape& s) const { return align256(ws_bytes(n, s)) + align256(s.pix * n); }

  void finish(Request* r, tok_status st) {
    r->status = st;
    r->state = Request::DONE;
    r->t_done = Clock::now();
    ++finished;
  }

  // Launch one batch on slot k.  Called with the lock held.
  tok_status launch(Batch* b, int k) {
    const Shape& s = b->reqs[0]->shape;
    const int n = (int)b->reqs.size();
    hipStream_t st = streams[k];
    char* ws = b->scratch;
    const size_t wsb = ws_bytes(n, s);
    uint8_t* pix = reinterpret_cast<uint8_t*>(ws + align256(wsb));
    for (int i = 0; i < n; ++i) {
      if (hipMemcpyAsync(pix + (size_t)i * s.pix, b->reqs[i]->req.pixels, s.pix, hipMemcpyHostToDevice, st) !=
          hipSuccess)
        return TOK_EDEVICE;
    }
    Request* r0 = b->reqs[0];
    float* codes = reinterpret_cast<float*>(r0->results);
    // A batch's results share one arena block laid out by kind: the codes of
    // all n clips, then their idx, keep and xhat; each clip gets views into it.
    const size_t cb = align256(s.tok * 6 * 4 * n), ib = align256(s.tok * 4 * n), kb = align256(s.tok * n);
    int32_t* idx = reinterpret_cast<int32_t*>(r0->results + cb);
    uint8_t* keep = reinterpret_cast<uint8_t*>(r0->results + cb + ib);
    float* xhat = reinterpret_cast<float*>(r0->results + cb + ib + kb);
    tok_status e = tok_encode(model, pix, n, s.T, s.H, s.W, nullptr, codes, idx, nullptr, nullptr, ws, wsb, st);
    if (e != TOK_OK) return e;
    for (int i = 0; i < n; ++i) {
      tok_drop_desc d = b->reqs[i]->req.drop;
      d.ext_keep = nullptr;
      float* ci = codes + (size_t)i * s.tok * 6;
      uint8_t* ki = keep + (size_t)i * s.tok;
      // the selection's scratch is the batch workspace, idle between encode and decode
      e = d.mode == TOK_DROP_SIMILARITY ? tok_select_similar(d.rate, ci, ki, 1, s.T2, s.H2, s.W2, ws, wsb, st)
                                         : tok_drop(&d, ci, ki, 1, s.T2, s.H2, s.W2, st);
      if (e != TOK_OK) return e;
    }
    e = tok_decode(model, codes, n, s.T2, s.H2, s.W2, xhat, ws, wsb, st);
    if (e != TOK_OK) return e;
    if (hipEventRecord(events[k], st) != hipSuccess) return TOK_EDEVICE;
    return TOK_OK;
  }

  // Try to admit the oldest queued request, batched with same-shape ones.
  bool admit_one() {
    int k = -1;
    for (size_t i = 0; i < slot_batch.size(); ++i)
      if (!slot_batch[i]) { k = (int)i; break; }
    if (k < 0 || queue.empty()) return false;
    // Admission is strictly first-in first-out: a batch is the head plus the
    // run of consecutive queued clips of the same shape.  A queued clip is then
    // never older than an admitted one, so a client that waits for results in
    // submission order and holds the results of later clips meanwhile can never
    // starve the clip it waits for of arena memory.
    Request* head = queue.front();
    std::vector<Request*> cand{head};
    for (size_t i = 1; i < queue.size() && (int)cand.size() < max_batch && queue[i]->shape == head->shape; ++i)
      cand.push_back(queue[i]);
    // largest batch that fits the arena now
    while (!cand.empty()) {
      const int n = (int)cand.size();
      char* scratch = arena.alloc(scratch_bytes(n, head->shape));
      char* res = scratch ? arena.alloc(result_bytes(head->shape) * n + 4096) : nullptr;
      if (scratch && res) {
        Batch* b = new Batch;
        b->reqs = cand;
        b->slot = k;
        b->scratch = scratch;
        const auto now = Clock::now();
        for (Request* r : cand) {
          r->state = Request::RUNNING;
          r->t_admit = now;
          r->batch_size = n;
          r->results = nullptr;
        }
        cand[0]->results = res;  // the batch's result block; clip views below
        for (Request* r : cand)
          for (auto it = queue.begin(); it != queue.end(); ++it)
            if (*it == r) { queue.erase(it); break; }
        const tok_status e = launch(b, k);
        if (e != TOK_OK) {
          hipStreamSynchronize(streams[k]);
          arena.release(scratch);
          arena.release(res);
          // the block is back in the arena: no request may keep a view of it
          // (a later release would free it again, a wait would hand out views
          // into whatever batch the arena gives it to next)
          for (Request* r : cand) r->results = nullptr;
          for (Request* r : cand) finish(r, e);
          delete b;
          cv.notify_all();
          return true;
        }
        slot_batch[k] = b;
        return true;
      }
      if (scratch) arena.release(scratch);
      cand.pop_back();
    }
    return false;
  }

  void complete(int k) {
    Batch* b = slot_batch[k];
    slot_batch[k] = nullptr;
    arena.release(b->scratch);
    const int n = (int)b->reqs.size();
    char* res = b->reqs[0]->results;
    // hand each clip its own views into the batch's result block; the block is
    // returned to the arena when the last clip of the batch is released
    for (int i = 0; i < n; ++i) {
      b->reqs[i]->results = res;
      finish(b->reqs[i], TOK_OK);
    }
    delete b;
  }

  void run() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      bool busy = false;
      for (size_t k = 0; k < slot_batch.size(); ++k) {
        if (!slot_batch[k]) continue;
        busy = true;
        const hipError_t q = hipEventQuery(events[k]);
        if (q == hipSuccess) complete((int)k);
        else if (q != hipErrorNotReady) {
          Batch* b = slot_batch[k];
          slot_batch[k] = nullptr;
          arena.release(b->scratch);
          for (Request* r : b->reqs) finish(r, TOK_EDEVICE);
          delete b;
        }
      }
      if (stop) {
        bool any = false;
        for (auto* b : slot_batch) any |= b != nullptr;
        if (!any) break;
      } else {
        while (admit_one()) {
        }
      }
      cv.notify_all();
      if (busy || !queue.empty()) cv.wait_for(lk, std::chrono::microseconds(50));
      else cv.wait_for(lk, std::chrono::milliseconds(5));
    }
    for (Request* r : queue) finish(r, TOK_EINVAL);
    queue.clear();
    cv.notify_all();
  }
};

namespace {
struct ResultView {
  const float* codes;
  const int32_t* idx;
  const uint8_t* keep;
  const float* xhat;
};

// Clip i's views into a batch result block of n clips.
ResultView views(char* res, const Shape& s, int n, int i) {
  const size_t cb = align256(s.tok * 6 * 4 * n), ib = align256(s.tok * 4 * n), kb = align256(s.tok * n);
  ResultView v;
  v.codes = reinterpret_cast<const float*>(res) + (size_t)i * s.tok * 6;
  v.idx = reinterpret_cast<const int32_t*>(res + cb) + (size_t)i * s.tok;
  v.keep = reinterpret_cast<const uint8_t*>(res + cb + ib) + (size_t)i * s.tok;
  v.xhat = reinterpret_cast<const float*>(res + cb + ib + kb) + (size_t)i * s.xhat;
  return v;
}
}  // namespace

extern "C" {

tok_status tok_server_request_bytes(const tok_model* model, int T, int H, int W, size_t* bytes) {
  Shape s;
  if (!model || !bytes) return TOK_EINVAL;
  if (!make_shape(T, H, W, &s)) return TOK_ESHAPE;
  size_t ws = 0;
  const tok_status e = tok_workspace_size(model, 1, T, H, W, TOK_WS_ROUNDTRIP | TOK_WS_STREAM, &ws);
  if (e != TOK_OK) return e;
  *bytes = align256(ws) + align256(s.pix) + result_bytes(s) + 4096;
  return TOK_OK;
}

tok_status tok_server_create(tok_model* model, size_t budget_bytes, int slots, int max_batch, tok_server** out) {
  if (!model || !out || slots < 1 || max_batch < 1 || budget_bytes < 4096) return TOK_EINVAL;
  size_t probe = 0;  // the server runs round trips: the model must support them
  const tok_status ps = tok_workspace_size(model, 1, 1, 4, 4, TOK_WS_ROUNDTRIP, &probe);
  if (ps != TOK_OK) return ps;
  tok_server* sv = new tok_server;
  sv->model = model;
  sv->max_batch = max_batch;
  hipGetDevice(&sv->device);
  if (hipMalloc(&sv->mem, budget_bytes) != hipSuccess) {
    delete sv;
    return TOK_ENOMEM;
  }
  sv->arena.init(sv->mem, budget_bytes);
  sv->streams.resize(slots);
  sv->events.resize(slots);
  sv->slot_batch.assign(slots, nullptr);
  for (int k = 0; k < slots; ++k) {
    if (hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sv->events[k], hipEventDisableTiming) != hipSuccess) {
      hipFree(sv->mem);
      delete sv;
      return TOK_EDEVICE;
    }
  }
  sv->worker = std::thread([sv] { sv->run(); });
  *out = sv;
  return TOK_OK;
}

tok_status tok_server_submit(tok_server* sv, const tok_request* req, uint64_t* ticket) {
  if (!sv || !req || !req->pixels || !ticket) return TOK_EINVAL;
  Shape s;
  if (!make_shape(req->T, req->H, req->W, &s)) return TOK_ESHAPE;
  // no external masks (the request does not outlive its pixels' upload)
  if (req->drop.mode < TOK_DROP_NONE || req->drop.mode > TOK_DROP_SIMILARITY || req->drop.mode == TOK_DROP_EXTERNAL)
    return TOK_EINVAL;
  Request* r = new Request;
  r->req = *req;
  r->shape = s;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->scratch_bytes(1, s) + result_bytes(s) + 8192 > sv->arena.size()) {
    delete r;
    return TOK_EBUDGET;
  }
  r->ticket = sv->next_ticket++;
  sv->reqs[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv.notify_all();
  return TOK_OK;
}

int tok_server_wait(tok_server* sv, uint64_t ticket, int timeout_ms, tok_result* out) {
  if (!sv || !out) return TOK_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return TOK_EINVAL;
  Request* r = it->second;
  auto done = [&] { return r->state == Request::DONE || r->state == Request::RELEASED; };
  if (timeout_ms < 0) sv->cv.wait(lk, done);
  else if (!sv->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) return 1;
  std::memset(out, 0, sizeof(*out));
  out->ticket = ticket;
  out->status = r->status;
  out->T2 = r->shape.T2; out->H2 = r->shape.H2; out->W2 = r->shape.W2;
  out->batch_size = r->batch_size;
  if (r->status == TOK_OK && r->state == Request::DONE) {
    // clip index inside its batch: a batch's clips were admitted in ticket order
    char* res = r->results;
    int i = 0;
    for (auto& kv : sv->reqs)
      if (kv.second->results == res && kv.second->ticket < ticket) ++i;
    const ResultView v = views(res, r->shape, r->batch_size, i);
    out->codes = v.codes; out->idx = v.idx; out->keep = v.keep; out->xhat = v.xhat;
  }
  out->queue_ms = ms_between(r->t_submit, r->t_admit);
  out->run_ms = ms_between(r->t_admit, r->t_done);
  out->total_ms = ms_between(r->t_submit, r->t_done);
  if (r->status != TOK_OK) out->queue_ms = out->run_ms = 0.0;
  return TOK_OK;
}

tok_status tok_server_copy_result(tok_server* sv, uint64_t ticket, float* codes, int32_t* idx, uint8_t* keep,
                                  float* xhat, hipStream_t stream) {
  tok_result r;
  const int w = tok_server_wait(sv, ticket, 0, &r);
  if (w != TOK_OK) return w > 0 ? TOK_EINVAL : (tok_status)w;
  if (r.status != TOK_OK) return r.status;
  Shape s;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end() || it->second->state != Request::DONE) return TOK_EINVAL;
    s = it->second->shape;
  }
  if (codes && hipMemcpyAsync(codes, r.codes, s.tok * 6 * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TOK_EDEVICE;
  if (idx && hipMemcpyAsync(idx, r.idx, s.tok * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess) return TOK_EDEVICE;
  if (keep && hipMemcpyAsync(keep, r.keep, s.tok, hipMemcpyDeviceToDevice, stream) != hipSuccess) return TOK_EDEVICE;
  if (xhat && hipMemcpyAsync(xhat, r.xhat, s.xhat * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TOK_EDEVICE;
  return TOK_OK;
}

tok_status tok_server_release(tok_server* sv, uint64_t ticket) {
  if (!sv) return TOK_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end() || it->second->state != Request::DONE) return TOK_EINVAL;
  Request* r = it->second;
  char* res = r->results;
  r->state = Request::RELEASED;
  bool last = true;
  if (res) {
    for (auto& kv : sv->reqs)
      if (kv.second->results == res && kv.second->state != Request::RELEASED) last = false;
  }
  if (res && last) {
    sv->arena.release(res);
    std::vector<uint64_t> gone;
    for (auto& kv : sv->reqs)
      if (kv.second->results == res) gone.push_back(kv.first);
    for (uint64_t t : gone) {
      delete sv->reqs[t];
      sv->reqs.erase(t);
    }
  } else if (!res) {
    delete r;
    sv->reqs.erase(it);
  }
  sv->cv.notify_all();
  return TOK_OK;
}

tok_status tok_server_stats(tok_server* sv, int* queued, int* running, int* finished, size_t* in_use,
                            size_t* peak) {
  if (!sv) return TOK_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  int run = 0;
  for (auto* b : sv->slot_batch)
    if (b) run += (int)b->reqs.size();
  if (queued) *queued = (int)sv->queue.size();
  if (running) *running = run;
  if (finished) *finished = sv->finished;
  if (in_use) *in_use = sv->arena.used();
  if (peak) *peak = sv->arena.peak();
  return TOK_OK;
}

void tok_server_destroy(tok_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  sv->worker.join();
  for (size_t k = 0; k < sv->streams.size(); ++k) {
    hipStreamSynchronize(sv->streams[k]);
    hipStreamDestroy(sv->streams[k]);
    hipEventDestroy(sv->events[k]);
  }
  for (auto& kv : sv->reqs) delete kv.second;
  hipFree(sv->mem);
  delete sv;
}

}  // extern "C"
