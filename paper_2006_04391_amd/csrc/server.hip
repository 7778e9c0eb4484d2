// server.hip -- continuous-batching service for material-point evaluation
// requests (uneven sizes, several load steps each, state kept on the
// device).
//
// Host side: a scheduler thread owns two HIP streams and one device arena
// of the memory budget. Requests are admitted in arrival order while their
// device block (phase ids, internal variables, stress: 97 B per point, plus
// the phase tables) fits in the arena (first-fit, coalescing). Every round
// builds one batch with the next load step of admitted requests (a ragged
// table of segments) and launches one kernel over all of them. Two rounds
// are in flight: the next batch is queued behind the running one (a
// request's next load step may follow its previous one, stream order keeps
// them apart) before the scheduler waits for the older one, so the device
// does not idle while the host retires a round and builds the next.
// Requests that arrived meanwhile are admitted by a second host thread and
// their inputs uploaded on a second stream (their first batch waits for an
// event; a batch leaves out requests whose uploads are still running while
// others are ready); the results of
// finished requests are copied on a third stream once their last batch is
// done, without waiting for the batch behind it. A
// batch takes the requests with the least remaining work first (points
// times load steps left) up to an optional point cap, with aging so that no
// request waits more than a few batches: small and nearly finished requests
// are not held behind large ones. Finished requests return their block at
// once. In sequential mode only one
// request is admitted at a time (one launch per load step, its load steps
// queued two deep like the batches), which is the per-request baseline.
//
// Device side: the batch kernel strides a resident grid over the 256-point
// tiles of all segments. A tile belongs to one segment: the block finds it
// from LDS-staged first-tile indices and keeps that request's descriptor and
// phase table in LDS. Each lane generates the step's strain for its point
// and loads a_n (in the first load step of a request without an initial
// state it takes a_n = 0 instead, and points without flow write those
// zeros, so the arena block needs no clearing at admission); points
// without flow are finished at once, flowing points
// are compacted into full waves (per-wave LDS queues, emptied before the
// block moves to another request) and run the same per-point solve as the
// plain evaluation kernel. Results therefore do not depend on what else is
// in the batch, except in the last bits: a wave decides together whether a
// trial point is evaluated to first order, and which points share a wave
// depends on the batch.
//
// Strain of load step j of K at point i: eps = (j / K) E_final + std z,
// z_c standard normal from Philox4x32-10 (Salmon, Moraes, Dror, Shaw 2011)
// keyed by the request seed with counter (i_lo, i_hi, j, w), w = 0, 1, and
// the Box-Muller transform of uniforms (u + 1/2) 2^-32: pairs (u0, u1),
// (u2, u3) of word 0 and (u0, u1) of word 1 give z_0 .. z_5.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "automat.h"
#include "gsm_kernel.hpp"
#include "host_common.hpp"

namespace automat {
namespace {

using Model = MSGSM;
using PC = PhaseConst<Model>;

struct Segment {
    const uint8_t *phase;
    double *a;
    double *sigma;
    const PC *tab;
    unsigned long long *nonconv;
    int64_t n;
    int64_t tile0;  // first batch tile of this segment
    double E[6];    // macro strain of this step
    double noise;
    double h, tol;
    uint32_t key0, key1;
    uint32_t step;
    int32_t max_iter;
    int32_t n_phases;
    int32_t a_zero;  // first load step of a request without an initial state:
                     // a_n = 0 is not read, and points without flow write it
};

static_assert(sizeof(Segment) % sizeof(double) == 0, "Segment is copied as doubles");

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32 with 10 rounds
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ double u01(uint32_t u) { return ((double)u + 0.5) * 0x1p-32; }

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &z0, double &z1) {
    const double t = -2.0 * fm::log(u01(a));  // > 0 for u in (0, 1)
    const double r = t * fm::rsqrt(t);
    double s, c;
    sincospi(2.0 * u01(b), &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// A request's phase tables at admission; also clears its failure counter.
__global__ void build_tables_kernel(const Model::Phase *raw, int nph, PC *out,
                                    unsigned long long *nonconv) {
    const int k = threadIdx.x;
    if (k < nph) build_phase_const<Model>(raw[k], out[k], false);
    if (k == 0) *nonconv = 0ull;
}

// Segments per launch: their first-tile indices are staged in LDS.
constexpr int kMaxSegs = 2048;
constexpr int kWaves = kBlock / 64;
// Per-wave ring of queued flowing points: eps, a_n [12][kRing] doubles,
// then the point index [kRing] (int64) and phase id [kRing] (int32).
constexpr int kRing = 128;
constexpr size_t kRingBytes =
    12 * kRing * sizeof(double) + kRing * (sizeof(int64_t) + sizeof(int32_t));

size_t serve_smem_bytes() {
    return kWaves * kRingBytes + AUTOMAT_MAX_PHASES * sizeof(PC) + sizeof(Segment) +
           (kMaxSegs + 1) * sizeof(int32_t);
}

// Solve queued points head .. head + cnt - 1 of the current segment and
// store their results (one lane per point).
__device__ __forceinline__ void serve_run_batch(const Segment &sg, const PC *tab, double *ring,
                                                const int64_t *ridx, const int32_t *rpid,
                                                uint32_t head, uint32_t cnt, int lane) {
    const uint32_t slot = (head + (uint32_t)lane) & (kRing - 1);
    const bool active = (uint32_t)lane < cnt;
    const int pid = active ? rpid[slot] : 0;
    const int64_t i = active ? ridx[slot] : 0;
    double sig[6], anew[6], D[6] = {0, 0, 0, 0, 0, 0};
    const int status = solve_point<Model, false, kRing>(tab[pid], active, ring + slot,
                                                        ring + 6 * kRing + slot, sg.h, sg.tol,
                                                        sg.max_iter, 0u, D, sig, anew, nullptr);
    if (active) {
        const int64_t n = sg.n;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            __builtin_nontemporal_store(sig[c], sg.sigma + c * n + i);
            sg.a[c * n + i] = anew[c];
        }
    }
    count_failures(sg.nonconv, active && status < 0);
    wave_lds_sync();
}

// One launch covers the next load step of every request in the batch. A
// block walks 256-point tiles; each tile belongs to one segment (request),
// whose descriptor and phase table the block keeps in LDS. Each wave takes
// the tile's 64-point quarter: points that do not flow are finished at
// once, flowing points are queued in the wave's ring and solved 64 at a
// time (compaction, as in the evaluation kernel). A wave's queue is emptied
// before its block moves to another segment, so a batch never mixes
// requests.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void serve_batch_kernel(const Segment *segs, const int32_t *starts, int nseg, int32_t total_tiles) {
    extern __shared__ double smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *ring = smem_raw + wave * (kRingBytes / sizeof(double));
    int64_t *ridx = reinterpret_cast<int64_t *>(ring + 12 * kRing);
    int32_t *rpid = reinterpret_cast<int32_t *>(ridx + kRing);
    PC *tab = reinterpret_cast<PC *>(smem_raw + kWaves * (kRingBytes / sizeof(double)));
    Segment *cur = reinterpret_cast<Segment *>(tab + AUTOMAT_MAX_PHASES);
    int32_t *first = reinterpret_cast<int32_t *>(cur + 1);  // [nseg + 1], last = total_tiles
    for (int k = threadIdx.x; k <= nseg; k += kBlock) first[k] = starts[k];
    __syncthreads();
    uint32_t head = 0, tail = 0;  // this wave's queue positions
    int seg = -1;
    for (int32_t t = blockIdx.x;; t += gridDim.x) {
        const bool more = t < total_tiles;
        // tiles of a block ascend, so the owning segment only moves forward;
        // every lane reads the same LDS words, the result is block-uniform
        int ns = seg;
        if (more) {
            ns = seg < 0 ? 0 : seg;
            while (first[ns + 1] <= t) ++ns;
        }
        if (ns != seg || !more) {
            // drain this wave's queue with the old segment's table
            if (seg >= 0 && tail != head) {
                serve_run_batch(*cur, tab, ring, ridx, rpid, head, tail - head, lane);
                head = tail;
            }
            if (!more) break;
            __syncthreads();  // every wave is done with the previous segment
            {
                const double *src = reinterpret_cast<const double *>(segs + ns);
                double *dst = reinterpret_cast<double *>(cur);
                for (int w = threadIdx.x; w < (int)(sizeof(Segment) / sizeof(double)); w += kBlock)
                    dst[w] = src[w];
                const int nph = segs[ns].n_phases;
                const double *tsrc = reinterpret_cast<const double *>(segs[ns].tab);
                double *tdst = reinterpret_cast<double *>(tab);
                const int words = nph * (int)(sizeof(PC) / sizeof(double));
                for (int w = threadIdx.x; w < words; w += kBlock) tdst[w] = tsrc[w];
            }
            __syncthreads();
            seg = ns;
        }
        const Segment &sg = *cur;
        const int64_t i = (int64_t)(t - sg.tile0) * kBlock + threadIdx.x;
        const bool in_range = i < sg.n;
        bool queue = false;
        double e[6], a[6];
        int pid = 0;
        if (in_range) {
            const U4 r0 = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), sg.step, 0u}, sg.key0,
                                        sg.key1);
            const U4 r1 = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), sg.step, 1u}, sg.key0,
                                        sg.key1);
            double z[6];
            box_muller(r0.x, r0.y, z[0], z[1]);
            box_muller(r0.z, r0.w, z[2], z[3]);
            box_muller(r1.x, r1.y, z[4], z[5]);
            const int64_t n = sg.n;
            bool finite_in = true;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e[c] = sg.E[c] + sg.noise * z[c];
                a[c] = sg.a_zero ? 0.0 : sg.a[c * n + i];
                finite_in = finite_in && isfinite(e[c]) && isfinite(a[c]);
            }
            pid = sg.phase[i];
            const bool valid = pid < sg.n_phases && finite_in;
            const PC &pc = tab[valid ? pid : 0];
            queue = valid && Model::flows(pc.prm);
            if (!queue) {
                // no flow: a_{n+1} = a_n stays in place
                double sig[6];
                if (valid) {
                    Model::stress(pc.prm, e, a, sig);
                    if (sg.a_zero) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) sg.a[c * n + i] = 0.0;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        sig[c] = NAN;
                        sg.a[c * n + i] = NAN;
                    }
                }
#pragma unroll
                // cached stores, so that the line merges in L2 with the
                // flowing points written one Newton batch later
                for (int c = 0; c < 6; ++c) sg.sigma[c * n + i] = sig[c];
            }
            count_failures(sg.nonconv, !valid);
        }
        const uint64_t mask = __ballot(queue);
        if (queue) {
            const uint32_t slot = (tail + lane_rank(mask)) & (kRing - 1);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                ring[c * kRing + slot] = e[c];
                ring[(6 + c) * kRing + slot] = a[c];
            }
            ridx[slot] = i;
            rpid[slot] = pid;
        }
        tail += (uint32_t)__popcll(mask);
        wave_lds_sync();
        if (tail - head >= 64) {
            serve_run_batch(sg, tab, ring, ridx, rpid, head, 64, lane);
            head += 64;
        }
    }
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t round_up(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit sub-allocator over one device arena (offsets only; blocks are
// 256-byte aligned, neighbours coalesce on release).
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            *off = o;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[off] = bytes;
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

// Device block of one request, in this order: phase ids, a (6 x n), sigma
// (6 x n), derived phase table, raw phase parameters, failure counter.
struct Layout {
    size_t phase, a, sigma, tab, raw, nonconv, total;
};

Layout layout_of(int64_t n, int nph) {
    Layout l;
    l.phase = 0;
    l.a = l.phase + round_up((size_t)n);
    l.sigma = l.a + round_up((size_t)n * 6 * sizeof(double));
    l.tab = l.sigma + round_up((size_t)n * 6 * sizeof(double));
    l.raw = l.tab + round_up((size_t)nph * sizeof(PC));
    l.nonconv = l.raw + round_up((size_t)nph * sizeof(Model::Phase));
    l.total = l.nonconv + 256;
    return l;
}

// Launch descriptor buffer for cap segments: the segments, then their
// first-tile indices (cap + 1 int32).
size_t seg_bytes(int cap) {
    return (size_t)cap * sizeof(Segment) + (size_t)(cap + 1) * sizeof(int32_t);
}

struct Req {
    uint64_t id = 0;
    automat_request r{};
    Model::Phase raw[AUTOMAT_MAX_PHASES];
    int32_t nph = 0;
    size_t off = 0;  // arena offset of the request's block
    Layout lay{};
    uint8_t *d_phase = nullptr;
    double *d_a = nullptr;
    double *d_sigma = nullptr;
    PC *d_tab = nullptr;
    Model::Phase *d_raw = nullptr;
    unsigned long long *d_nonconv = nullptr;
    hipEvent_t ready = nullptr;  // uploads and table build done
    int32_t steps_done = 0;      // load steps of retired batches
    int32_t steps_launched = 0;  // load steps of launched batches
    bool a_zero = false;         // no initial state: the first step takes a_n = 0
    int64_t last_round = 0;      // round of the last batch that took a step of it
    double t_arrival = 0, t_admit = 0, t_done = 0;
    int32_t status = 0;
};

}  // namespace
}  // namespace automat

using namespace automat;

struct automat_server {
    size_t budget = 0, used = 0;
    int64_t max_batch_points = 0;
    int sequential = 0;
    int device = 0;
    int grid = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> pending;
    std::vector<Req *> active;
    std::deque<automat_result> done;
    std::thread worker;
    std::thread uploader;        // admissions: arena blocks and input uploads
    int64_t uploading = 0;       // admitted requests whose uploads are being queued
    bool blocked = false;        // the next request in line does not fit the arena
    uint64_t gen = 0;            // bumped by submissions and retirements
    bool stop = false;
    uint64_t next_id = 1;
    std::chrono::steady_clock::time_point t0;
    hipStream_t stream = nullptr;  // batch kernels
    hipStream_t up = nullptr;      // admissions: uploads and table builds
    hipStream_t down = nullptr;    // result copies of finished requests
    char *arena_base = nullptr;
    Arena arena;
    // per round slot (two rounds in flight): segment tables, timing events
    Segment *d_segs[2] = {nullptr, nullptr}, *h_segs[2] = {nullptr, nullptr};
    int seg_cap[2] = {0, 0};
    hipEvent_t ev_start[2] = {nullptr, nullptr}, ev_end[2] = {nullptr, nullptr};
    int64_t round = 0;  // batches built so far
    // statistics
    int64_t launches = 0, updates = 0;
    double busy_s = 0;
};

// Under s->mu: take requests from the head of the queue while their blocks
// fit in the arena (arrival order, no overtaking); they join the active set
// once their uploads are queued.
static void take_admissible(automat_server *s, std::vector<Req *> &fresh) {
    const size_t max_active = s->sequential ? 1 : (size_t)1 << 20;
    s->blocked = false;
    while (!s->stop && !s->pending.empty() &&
           s->active.size() + (size_t)s->uploading < max_active) {
        Req *q = s->pending.front();
        if (!s->arena.alloc(q->lay.total, &q->off)) {
            s->blocked = true;
            break;
        }
        s->pending.pop_front();
        q->last_round = s->round;
        s->used += q->lay.total;
        s->uploading += 1;
        fresh.push_back(q);
    }
}

// Retire a request: copy its results (status OK: after the event `after`,
// which marks its last batch, on the copy stream), return its block.
static void finish(automat_server *s, Req *q, int32_t status, hipEvent_t after = nullptr) {
    unsigned long long nc = 0;
    if (status == AUTOMAT_OK) {
        bool ok = !after || hipStreamWaitEvent(s->down, after, 0) == hipSuccess;
        if (q->r.sigma_host)
            ok = ok && hipMemcpyAsync(q->r.sigma_host, q->d_sigma, (size_t)q->r.n * 6 * sizeof(double),
                                      hipMemcpyDeviceToHost, s->down) == hipSuccess;
        if (q->r.a_host)
            ok = ok && hipMemcpyAsync(q->r.a_host, q->d_a, (size_t)q->r.n * 6 * sizeof(double),
                                      hipMemcpyDeviceToHost, s->down) == hipSuccess;
        ok = ok && hipMemcpyAsync(&nc, q->d_nonconv, sizeof nc, hipMemcpyDeviceToHost, s->down) ==
                       hipSuccess;
        ok = ok && hipStreamSynchronize(s->down) == hipSuccess;
        if (!ok) status = AUTOMAT_EHIP;
    } else if (q->ready) {
        // the block may still be written by an upload: let it drain first
        (void)hipEventSynchronize(q->ready);
    }
    if (q->ready) (void)hipEventDestroy(q->ready);
    q->ready = nullptr;
    q->status = status;
    q->t_done = now_s(s->t0);
    automat_result res{};
    res.id = q->id;
    res.status = status;
    res.steps_done = q->steps_done;
    res.n = q->r.n;
    res.nonconverged = (int64_t)nc;
    res.t_arrival = q->t_arrival;
    res.t_admit = q->t_admit;
    res.t_done = q->t_done;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = std::find(s->active.begin(), s->active.end(), q);
    if (it != s->active.end()) s->active.erase(it);
    s->gen += 1;
    s->arena.release(q->off, q->lay.total);
    s->used -= q->lay.total;
    s->done.push_back(res);
    delete q;
    s->cv.notify_all();
}

// Queue the uploads of a freshly admitted request on the admission stream;
// its first batch waits for the recorded event.
static int32_t start_upload(automat_server *s, Req *q) {
    char *b = s->arena_base + q->off;
    const int64_t n = q->r.n;
    q->d_phase = reinterpret_cast<uint8_t *>(b + q->lay.phase);
    q->d_a = reinterpret_cast<double *>(b + q->lay.a);
    q->d_sigma = reinterpret_cast<double *>(b + q->lay.sigma);
    q->d_tab = reinterpret_cast<PC *>(b + q->lay.tab);
    q->d_raw = reinterpret_cast<Model::Phase *>(b + q->lay.raw);
    q->d_nonconv = reinterpret_cast<unsigned long long *>(b + q->lay.nonconv);
    q->t_admit = now_s(s->t0);
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) {
        q->ready = nullptr;
        return AUTOMAT_EHIP;
    }
    const size_t abytes = (size_t)n * 6 * sizeof(double);
    // without an initial state the first load step writes a_n = 0 itself
    q->a_zero = q->r.a_init == nullptr;
    bool ok = hipMemcpyAsync(q->d_phase, q->r.phase, (size_t)n, hipMemcpyHostToDevice, s->up) ==
                  hipSuccess &&
              (!q->r.a_init || hipMemcpyAsync(q->d_a, q->r.a_init, abytes,
                                              hipMemcpyHostToDevice, s->up) == hipSuccess) &&
              hipMemcpyAsync(q->d_raw, q->raw, (size_t)q->nph * sizeof(Model::Phase),
                             hipMemcpyHostToDevice, s->up) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(build_tables_kernel, dim3(1), dim3(64), 0, s->up, q->d_raw, q->nph,
                           q->d_tab, q->d_nonconv);
        ok = hipGetLastError() == hipSuccess && hipEventRecord(q->ready, s->up) == hipSuccess;
    }
    return ok ? AUTOMAT_OK : AUTOMAT_EHIP;
}

static void admit(automat_server *s, std::vector<Req *> &fresh) {
    // the smallest first: their inputs arrive first and the first batches
    // (least remaining work first) need them
    std::stable_sort(fresh.begin(), fresh.end(), [](const Req *a, const Req *b) {
        return a->r.n * (int64_t)a->r.steps < b->r.n * (int64_t)b->r.steps;
    });
    for (Req *q : fresh) {
        const int32_t rc = start_upload(s, q);
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->uploading -= 1;
            if (rc == AUTOMAT_OK) s->active.push_back(q);
        }
        if (rc != AUTOMAT_OK) finish(s, q, rc);
        s->cv.notify_all();
    }
    fresh.clear();
}

// The admission thread: takes the requests that fit and queues their
// uploads (from pageable host memory these copies can block the calling
// thread, so they stay off the batch scheduler's thread).
static void uploader_loop(automat_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<Req *> fresh;
    uint64_t seen = ~(uint64_t)0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv.wait(lock, [&] { return s->stop || s->gen != seen; });
            if (s->stop) return;
            seen = s->gen;
            take_admissible(s, fresh);
        }
        admit(s, fresh);
    }
}

// batches a request may be left out of before it goes first
constexpr int64_t kAging = 16;
// point cap multiplier while the next request waits for arena space
constexpr int64_t kSaturatedCap = 4;

// a launched batch that is not retired yet
struct Round {
    std::vector<Req *> batch;
    int slot = 0;
    bool ok = true;
};

static bool ensure_segs(automat_server *s, int slot, int need) {
    if (need <= s->seg_cap[slot]) return true;
    if (s->d_segs[slot]) (void)hipFree(s->d_segs[slot]);
    if (s->h_segs[slot]) (void)hipHostFree(s->h_segs[slot]);
    const int cap = std::min<int>(kMaxSegs, std::max<int>(need, 2 * s->seg_cap[slot]));
    if (hipMalloc(&s->d_segs[slot], seg_bytes(cap)) != hipSuccess ||
        hipHostMalloc(&s->h_segs[slot], seg_bytes(cap), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->seg_cap[slot] = 0;
        s->d_segs[slot] = nullptr;
        s->h_segs[slot] = nullptr;
        return false;
    }
    s->seg_cap[slot] = cap;
    return true;
}

// Build the next batch from the active requests with load steps left to
// launch. Latency-aware order: the least remaining work (points x steps not
// launched) first, so that small and nearly finished requests are not held
// behind large ones; a request left out of kAging consecutive batches goes
// first. The point cap admits at least one request.
static void build_batch(automat_server *s, std::vector<Req *> &order, std::vector<Req *> &batch) {
    batch.clear();
    std::lock_guard<std::mutex> lock(s->mu);
    order.clear();
    // requests whose inputs are still being uploaded wait for a later batch
    // while others are ready (a batch would otherwise stall on their upload)
    for (Req *q : s->active)
        if (q->steps_launched < q->r.steps &&
            (q->steps_launched > 0 || hipEventQuery(q->ready) == hipSuccess))
            order.push_back(q);
    if (order.empty()) {
        for (Req *q : s->active)
            if (q->steps_launched < q->r.steps) order.push_back(q);
    }
    if (order.empty()) return;
    const int64_t rnd = ++s->round;
    auto starved = [&](const Req *q) { return rnd - q->last_round > kAging; };
    auto remaining = [](const Req *q) { return q->r.n * (int64_t)(q->r.steps - q->steps_launched); };
    std::stable_sort(order.begin(), order.end(), [&](const Req *a, const Req *b) {
        if (starved(a) != starved(b)) return starved(a);
        return remaining(a) < remaining(b);
    });
    // While requests wait in the queue (for arena space, or for the
    // admission thread) the device is saturated and larger batches (fewer
    // launches) pay; otherwise the cap keeps batches short, so that a
    // request arriving meanwhile does not wait behind a long one.
    const bool backlog = s->blocked || !s->pending.empty();
    const int64_t cap = backlog ? kSaturatedCap * s->max_batch_points : s->max_batch_points;
    int64_t pts = 0;
    for (Req *q : order) {
        if (batch.size() >= (size_t)kMaxSegs) break;
        if (!batch.empty() && cap > 0 && pts + q->r.n > cap) continue;
        batch.push_back(q);
        pts += q->r.n;
        q->last_round = rnd;
    }
}

// Queue one batch (segment table upload and kernel) on the batch stream
// between the slot's timing events.
static bool launch_round(automat_server *s, Round &r) {
    const int slot = r.slot;
    if (!ensure_segs(s, slot, (int)r.batch.size())) return false;
    Segment *hs = s->h_segs[slot];
    int64_t tiles = 0;
    bool ok = hipEventRecord(s->ev_start[slot], s->stream) == hipSuccess;
    for (size_t k = 0; k < r.batch.size(); ++k) {
        Req *q = r.batch[k];
        if (q->steps_launched == 0)
            ok = ok && hipStreamWaitEvent(s->stream, q->ready, 0) == hipSuccess;
        Segment &g = hs[k];
        g.phase = q->d_phase;
        g.a = q->d_a;
        g.sigma = q->d_sigma;
        g.tab = q->d_tab;
        g.nonconv = q->d_nonconv;
        g.n = q->r.n;
        g.tile0 = tiles;
        const int32_t step = q->steps_launched + 1;
        for (int c = 0; c < 6; ++c) g.E[c] = q->r.E_final[c] * ((double)step / q->r.steps);
        g.noise = q->r.noise_std;
        g.h = q->r.h;
        g.tol = q->r.tol;
        g.key0 = (uint32_t)q->r.seed;
        g.key1 = (uint32_t)(q->r.seed >> 32);
        g.step = (uint32_t)step;
        g.max_iter = q->r.max_iter;
        g.n_phases = q->nph;
        g.a_zero = q->a_zero && q->steps_launched == 0;
        tiles += (q->r.n + kBlock - 1) / kBlock;
    }
    const int nseg = (int)r.batch.size();
    int32_t *h_first = reinterpret_cast<int32_t *>(hs + s->seg_cap[slot]);
    for (int k = 0; k < nseg; ++k) h_first[k] = (int32_t)hs[k].tile0;
    h_first[nseg] = (int32_t)tiles;
    int32_t *d_first = reinterpret_cast<int32_t *>(s->d_segs[slot] + s->seg_cap[slot]);
    ok = ok && tiles < INT32_MAX &&
         hipMemcpyAsync(s->d_segs[slot], hs, nseg * sizeof(Segment), hipMemcpyHostToDevice,
                        s->stream) == hipSuccess &&
         hipMemcpyAsync(d_first, h_first, (nseg + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                        s->stream) == hipSuccess;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)s->grid);
    if (ok) {
        hipLaunchKernelGGL(serve_batch_kernel, dim3(grid), dim3(kBlock), serve_smem_bytes(),
                           s->stream, s->d_segs[slot], d_first, nseg, (int32_t)tiles);
        ok = hipGetLastError() == hipSuccess;
    }
    ok = ok && hipEventRecord(s->ev_end[slot], s->stream) == hipSuccess;
    for (Req *q : r.batch) q->steps_launched += 1;
    return ok;
}

// Wait for the oldest round and retire it: its requests have one more load
// step done; those with all steps done are finished (results copied after
// the round's end event, not after the round queued behind it).
static void retire_round(automat_server *s, std::deque<Round> &inflight) {
    Round r = std::move(inflight.front());
    inflight.pop_front();
    bool ok = r.ok && hipEventSynchronize(s->ev_end[r.slot]) == hipSuccess;
    float ms = 0.0f;
    if (ok && hipEventElapsedTime(&ms, s->ev_start[r.slot], s->ev_end[r.slot]) == hipSuccess)
        s->busy_s += 1e-3 * ms;
    s->launches += 1;
    if (!ok) {
        // drain everything queued, then fail every request of every round
        // in flight once
        (void)hipStreamSynchronize(s->stream);
        std::vector<Req *> all(r.batch);
        for (Round &o : inflight) all.insert(all.end(), o.batch.begin(), o.batch.end());
        inflight.clear();
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        for (Req *q : all) finish(s, q, AUTOMAT_EHIP);
        return;
    }
    for (Req *q : r.batch) {
        q->steps_done += 1;
        s->updates += q->r.n;
        if (q->steps_done >= q->r.steps) finish(s, q, AUTOMAT_OK, s->ev_end[r.slot]);
    }
}

constexpr int kInFlight = 2;

static void worker_loop(automat_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<Req *> order;
    std::deque<Round> inflight;
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(s->mu);
            if (inflight.empty())
                s->cv.wait(lock, [&] {
                    return !s->active.empty() || (s->stop && s->uploading == 0);
                });
            if (s->stop && s->active.empty() && s->uploading == 0 && inflight.empty()) {
                for (Req *q : s->pending) {
                    automat_result res{};
                    res.id = q->id;
                    res.status = AUTOMAT_EINVAL;
                    res.t_arrival = q->t_arrival;
                    res.t_done = now_s(s->t0);
                    s->done.push_back(res);
                    delete q;
                }
                s->pending.clear();
                return;
            }
        }
        bool launched = false;
        if ((int)inflight.size() < kInFlight) {
            Round r;
            build_batch(s, order, r.batch);
            if (!r.batch.empty()) {
                r.slot = inflight.empty() ? 0 : 1 - inflight.back().slot;
                r.ok = launch_round(s, r);
                inflight.push_back(std::move(r));
                launched = true;
            }
        }
        if (!inflight.empty() && ((int)inflight.size() >= kInFlight || !launched))
            retire_round(s, inflight);
    }
}

extern "C" int32_t automat_server_create(size_t hbm_budget_bytes, int64_t max_batch_points,
                                         int32_t sequential, automat_server **out) {
    if (!out || hbm_budget_bytes < 4096 || max_batch_points < 0) return AUTOMAT_EINVAL;
    *out = nullptr;
    automat_server *s = new (std::nothrow) automat_server();
    if (!s) return AUTOMAT_ENOMEM;
    s->budget = hbm_budget_bytes & ~(size_t)255;
    s->max_batch_points = max_batch_points;
    s->sequential = sequential ? 1 : 0;
    s->t0 = std::chrono::steady_clock::now();
    int cus = 0;
    int32_t rc = AUTOMAT_OK;
    if (hipGetDevice(&s->device) != hipSuccess || device_cus(&cus) != AUTOMAT_OK ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->down, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev_start[0]) != hipSuccess || hipEventCreate(&s->ev_start[1]) != hipSuccess ||
        hipEventCreate(&s->ev_end[0]) != hipSuccess || hipEventCreate(&s->ev_end[1]) != hipSuccess)
        rc = AUTOMAT_EHIP;
    else if (hipMalloc(&s->arena_base, s->budget) != hipSuccess)
        rc = AUTOMAT_ENOMEM;
    if (rc != AUTOMAT_OK) {
        (void)hipGetLastError();
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->up) (void)hipStreamDestroy(s->up);
        if (s->down) (void)hipStreamDestroy(s->down);
        for (int k = 0; k < 2; ++k) {
            if (s->ev_start[k]) (void)hipEventDestroy(s->ev_start[k]);
            if (s->ev_end[k]) (void)hipEventDestroy(s->ev_end[k]);
        }
        delete s;
        return rc;
    }
    s->arena.reset(s->budget);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, serve_batch_kernel, kBlock,
                                                     serve_smem_bytes()) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    s->grid = cus * per_cu;
    s->worker = std::thread(worker_loop, s);
    s->uploader = std::thread(uploader_loop, s);
    *out = s;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_server_submit(automat_server *s, const automat_request *req,
                                         uint64_t *id) {
    if (!s || !req || !id) return AUTOMAT_EINVAL;
    if (req->n < 1 || !req->phase || req->steps < 1 || req->max_iter < 1) return AUTOMAT_EINVAL;
    if (!std::isfinite(req->h) || !(req->h > 0.0) || !(req->tol > 0.0) || !(req->noise_std >= 0.0))
        return AUTOMAT_EINVAL;
    Req *q = new (std::nothrow) Req();
    if (!q) return AUTOMAT_ENOMEM;
    q->r = *req;
    const int32_t rc = copy_params(&req->params, q->raw, &q->nph);
    if (rc) {
        delete q;
        return rc;
    }
    q->lay = layout_of(req->n, q->nph);
    if (q->lay.total > s->budget) {
        delete q;
        return AUTOMAT_EBUDGET;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) {
        delete q;
        return AUTOMAT_EINVAL;
    }
    q->id = s->next_id++;
    q->t_arrival = req->t_arrival >= 0.0 ? req->t_arrival : now_s(s->t0);
    s->pending.push_back(q);
    s->gen += 1;
    *id = q->id;
    s->cv.notify_all();
    return AUTOMAT_OK;
}

extern "C" int32_t automat_server_poll(automat_server *s, automat_result *out, int32_t max,
                                       int32_t *count) {
    if (!s || !count || (max > 0 && !out)) return AUTOMAT_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *count = k;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_server_stats(automat_server *s, automat_server_stats_t *st) {
    if (!s || !st) return AUTOMAT_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    st->clock_s = now_s(s->t0);
    st->pending = (int64_t)s->pending.size();
    st->active = (int64_t)s->active.size();
    st->used_bytes = (int64_t)s->used;
    st->launches = s->launches;
    st->updates = s->updates;
    st->busy_s = s->busy_s;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_server_destroy(automat_server *s) {
    if (!s) return AUTOMAT_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->uploader.joinable()) s->uploader.join();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->up);
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->down);
    for (Req *q : s->active) {
        if (q->ready) (void)hipEventDestroy(q->ready);
        delete q;
    }
    for (int k = 0; k < 2; ++k) {
        if (s->d_segs[k]) (void)hipFree(s->d_segs[k]);
        if (s->h_segs[k]) (void)hipHostFree(s->h_segs[k]);
        if (s->ev_start[k]) (void)hipEventDestroy(s->ev_start[k]);
        if (s->ev_end[k]) (void)hipEventDestroy(s->ev_end[k]);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->up) (void)hipStreamDestroy(s->up);
    if (s->down) (void)hipStreamDestroy(s->down);
    delete s;
    return AUTOMAT_OK;
}
