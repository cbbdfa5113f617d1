// bbfmm_matvec_static: the product of bbfmm_matvec without any device
// allocation, for callers that cannot allocate (tight serving loops,
// harnesses that forbid allocation).  Every buffer the product needs beyond
// its inputs and outputs -- sigma in tree order, the multipole and local
// expansions and their compressed forms, the M2L partials, the launch lists
// and tile masks -- is carved out of one fixed device array, `scratch`, in
// the order a plan would allocate them.
//
// The array is a file-scope __device__ object, so each GPU holds its own
// copy (at its own address) from the moment the library's code object is
// loaded on that GPU until the process ends.  Its device address is looked
// up once per device with hipGetSymbolAddress and used everywhere host code
// hands the memory to a kernel; the name itself is not a device address on
// the host.
//
// Every call on one GPU uses the same array and leaves it as the call's
// kernels wrote it; nothing in the array is read before the same call
// writes it (the gather, the up/down kernels and the M2L write every element
// of their outputs, zero padding included), so no clearing is needed.  The
// call is synchronous: it returns after the product, so consecutive calls
// from one thread never overlap.  Calls that overlap on one GPU (from
// several threads) race on the array.
#include <map>
#include <mutex>

#include "common.h"

namespace bbfmm {
namespace {

constexpr size_t kScratchBytes = BBFMM_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void *> g_addr;    // device -> address of its copy of `scratch`

void *scratch_address() {
    int dev = 0;
    BB_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_addr.find(dev);
    if (it != g_addr.end()) return it->second;
    void *p = nullptr;
    BB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BB_INTERNAL(p != nullptr, "no device address for the scratch array");
    g_addr[dev] = p;
    return p;
}

// Bump allocation from the array (256-byte aligned); freeing is a no-op.
struct Bump {
    char *base = nullptr;
    size_t cap = 0, used = 0, wanted = 0;
};

void *bump_alloc(size_t bytes, void *, void *ctx) {
    Bump &b = *static_cast<Bump *>(ctx);
    const size_t off = (b.used + 255) & ~size_t(255);
    b.wanted = off + bytes;
    if (b.wanted > b.cap) return nullptr;
    b.used = off + bytes;
    return b.base + off;
}

void bump_free(void *, void *, void *) {}

}  // namespace
}  // namespace bbfmm

using namespace bbfmm;

extern "C" bbfmm_status bbfmm_matvec_static(const bbfmm_tree *t, const bbfmm_ops *o,
                                            const float *sigma, int64_t r, float *phi,
                                            void *stream) {
    clear_error();
    try {
        BB_REQUIRE(t != nullptr && o != nullptr, "tree or ops is NULL");
        BB_REQUIRE(o->tree == t, "operators were built for another tree");
        BB_REQUIRE(sigma != nullptr && phi != nullptr, "sigma / phi is NULL");
        BB_REQUIRE(r >= 1 && r <= 4096, "r must be in [1, 4096]");
        hipStream_t s = static_cast<hipStream_t>(stream);
        Bump bump;
        bump.base = static_cast<char *>(scratch_address());
        bump.cap = kScratchBytes;
        const bbfmm_allocator hook{bump_alloc, bump_free, &bump};
        Plan *plan = nullptr;
        {
            MemScope scope(&hook, s);
            try {
                plan = plan_create_impl(t, o, r, nullptr, s, /*transient=*/true);
            } catch (const Exception &e) {
                if (e.status == BBFMM_ERR_OUT_OF_MEMORY && bump.wanted > bump.cap)
                    fail(BBFMM_ERR_INVALID_ARG,
                         "bbfmm_matvec_static: this product needs more than the %zu bytes of "
                         "fixed scratch (N = %lld, r = %lld)",
                         kScratchBytes, (long long)t->n, (long long)r);
                throw;
            }
        }
        struct Del {
            void operator()(Plan *q) const { plan_destroy(q); }
        };
        std::unique_ptr<Plan, Del> hold(plan);
        plan_execute_impl(plan, sigma, phi, s);
        // the plan's host-side launch lists are read by copies on s, and the
        // next call reuses the array: return once the product is done
        BB_HIP(hipStreamSynchronize(s));
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    } catch (...) {
        return BBFMM_ERR_INTERNAL;
    }
}
