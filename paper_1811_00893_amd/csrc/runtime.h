// Host runtime: contexts, resident gauge fields, device memory, event timing, the
// launch-configuration autotuner and error plumbing.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.h"
#include "wilson.h"

namespace wl {

// Internal error carrying a wilson_status; converted to a return code at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &m);
const std::string &last_error();
[[noreturn]] void hip_fail(hipError_t e, const char *what, const char *file, int line);
#define WL_HIP(x)                                                 \
    do {                                                          \
        hipError_t _e = (x);                                      \
        if (_e != hipSuccess) ::wl::hip_fail(_e, #x, __FILE__, __LINE__); \
    } while (0)
#define WL_CHECK_ARG(cond, msg)                                   \
    do {                                                          \
        if (!(cond)) throw ::wl::Error(WILSON_INVALID_ARG, msg);  \
    } while (0)

// Owning device allocation.
class DevBuf {
   public:
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { alloc(bytes); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
        return *this;
    }
    void alloc(size_t bytes);
    void release();
    void *get() const { return p_; }
    size_t size() const { return n_; }
    template <typename T>
    T *as() const { return reinterpret_cast<T *>(p_); }

   private:
    void *p_ = nullptr;
    size_t n_ = 0;
};

// Owning pinned host allocation, mapped into the device address space.
class PinnedBuf {
   public:
    PinnedBuf() = default;
    ~PinnedBuf();
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    void alloc(size_t bytes);
    void *host() const { return h_; }
    void *dev() const { return d_; }
    size_t size() const { return n_; }

   private:
    void *h_ = nullptr;
    void *d_ = nullptr;
    size_t n_ = 0;
};

bool is_device_ptr(const void *p);

// Host-side resources of one solve besides device memory: pinned, device-mapped per-RHS
// state records (a ring of mirrors the host polls, one upload and one read buffer) and the
// ring's events, for up to nrhs right-hand sides.
struct SolveHostRes {
    PinnedBuf mirror, hinit, hread;
    hipEvent_t ring[kStateRing] = {};
    int cap = 0;  // right-hand sides the buffers hold
    void create(int nrhs);
    ~SolveHostRes();
};

}  // namespace wl

struct wilson_gauge {
    wl::Geom g;
    int32_t dims[4];
    wl::DevBuf U[3];  // per wl::Prec
    int recon = 18;   // 12: links stored as two rows (SU(3) verified at upload)
    // clover term (optional): packed T = 1 + F and T^-1 for both parities, FP64 and FP32
    wl::DevBuf clovT[2], clovTi[2];
    size_t bytes() const {
        return U[0].size() + U[1].size() + U[2].size() + clovT[0].size() + clovT[1].size() + clovTi[0].size() +
               clovTi[1].size();
    }
    const void *links(int prec) const { return U[prec].get(); }
    bool has_clover() const { return clovT[0].get() != nullptr; }
    // blocks of parity par for spinors of precision prec (FP64 blocks for FP64, FP32 otherwise)
    const void *clover(bool inverse, int prec, int par) const {
        const int cp = prec == wl::P64 ? wl::P64 : wl::P32;
        const wl::DevBuf &b = inverse ? clovTi[cp] : clovT[cp];
        if (!b.get()) return nullptr;
        return static_cast<const char *>(b.get()) + (size_t)par * wl::clover_parity_bytes(cp, g);
    }
};

// Hop launch configurations chosen by the autotuner, shared by every context of the
// process (a configuration is a property of the device and the launch shape).
//   WILSON_TUNE=0                       no tuning: built-in default configuration
//   WILSON_HOP_CFG="block,rpt,xcd,zblk[,lds_kb[,wsplit[,shx[,dsplit[,ldsl[,tm]]]]]]"   pin every hop launch of a context
//                                       created after it is set (tests)
//   WILSON_TUNE_CACHE=path              JSON lines read at start, new entries appended
//   WILSON_TUNE_VERBOSE=1               print every timed candidate
struct TuneTable {
    std::mutex mu;
    std::map<std::string, wl::LaunchCfg> cfg;
    bool enabled = true;
    std::string path;
    void save(const std::string &key, const wl::LaunchCfg &c, double ms);
};
TuneTable &tune_table();

struct wilson_ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    // ---- event timing ----
    bool timing = false;
    struct Pending {
        hipEvent_t a, b;
        int cls;
        double bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    // pinned hop configuration (WILSON_HOP_CFG), read at the context's first hop launch
    bool cfg_read = false;
    bool forced = false;
    wl::LaunchCfg forced_cfg;
    // configurations already looked up by this context, keyed by launch shape (no string
    // building and no lock on the per-launch path)
    struct HotKey {
        int sp, gp, rc, rhs, L[4];
        bool operator==(const HotKey &o) const {
            return sp == o.sp && gp == o.gp && rc == o.rc && rhs == o.rhs && L[0] == o.L[0] && L[1] == o.L[1] &&
                   L[2] == o.L[2] && L[3] == o.L[3];
        }
    };
    std::vector<std::pair<HotKey, wl::LaunchCfg>> hot;
    double t_ms[WILSON_KERNEL_COUNT] = {0, 0};
    int64_t launches[WILSON_KERNEL_COUNT] = {0, 0};
    double t_bytes[WILSON_KERNEL_COUNT] = {0, 0};
    int64_t hop_launch_count = 0;  // always counted
    double bytes_issued = 0.0;     // algorithmic bytes of hop, vector and block kernels launched
    double flops_issued = 0.0;     // operator flops of the hops launched

    hipEvent_t get_event();
    void drain_timing();  // resolves pending event pairs (waits for them)


    // ---- scratch ----
    // host resources lent to solves whose device memory the caller provides (created with
    // the context, so those solves allocate nothing themselves)
    wl::SolveHostRes lend;
    void *scratch = nullptr;         // device address of the no-allocation solve's array on this device
    hipStream_t capture_stream = nullptr;  // stream that iteration chunks are captured on (HIP graphs)
    bool no_tune = false;            // set for the duration of a call that must not tune
    wl::DevBuf stage_in, stage_out;  // canonical staging for host pointers
    wl::DevBuf flag;                 // device int for finiteness checks
    wl::PinnedBuf pinned;            // small host mirror
    // cached workspaces: the last dslash shape, and up to 4 solve shapes (LRU)
    std::shared_ptr<void> dslash_ws;
    std::string dslash_key;
    std::vector<std::pair<std::string, std::shared_ptr<void>>> solve_cache;
    void *stage(wl::DevBuf &b, size_t bytes);
};

namespace wl {

// Launch a parity hop with the tuned configuration, timed if timing is on.
// algorithmic_bytes is the per-launch byte count used for achieved-bandwidth figures.
// Returns the number of blocks launched (the row length of the partials it wrote).
int hop(wilson_ctx *ctx, HopArgs &a, double algorithmic_bytes);
// Launch a BLAS kernel (timed as class BLAS).
void blas(wilson_ctx *ctx, int op, BlasArgs &a, double algorithmic_bytes);
// Launch any kernel sequence through `launch` (returning hipError_t), timed as class cls.
template <typename F>
void timed_launch(wilson_ctx *ctx, int cls, double algorithmic_bytes, F &&launch) {
    ctx->bytes_issued += algorithmic_bytes;
    if (ctx->timing) {
        hipEvent_t e0 = ctx->get_event(), e1 = ctx->get_event();
        WL_HIP(hipEventRecord(e0, ctx->stream));
        WL_HIP(launch());
        WL_HIP(hipEventRecord(e1, ctx->stream));
        ctx->pending.push_back({e0, e1, cls, algorithmic_bytes});
    } else {
        WL_HIP(launch());
    }
}
// Size of a partials buffer (doubles) that any hop or BLAS launch on g with nrhs can use.
size_t partials_doubles(const Geom &g, int nrhs);
// Algorithmic bytes of one hop launch (per output site: 8 links + input + output (+ y, z, w)).
double hop_bytes(const HopArgs &a);
// host replay of the kernels' site indexing on one lattice (indexcheck.cpp): the number
// of violations, the first described in `first`
long long index_check(const int32_t dims[4], std::string &first);

}  // namespace wl
