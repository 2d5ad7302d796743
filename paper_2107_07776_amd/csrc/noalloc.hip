// Library-owned static device scratch for the entry point that allocates
// nothing (tbdg_solve_pressure_noalloc).  The array lives in the code object:
// every GPU the library runs on holds its own copy from module load until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in symbol); it takes the device address from
// hipGetSymbolAddress once per device, with that device current, and uses
// that address everywhere.
#include <mutex>

#include "internal.hpp"

namespace trbdg {

namespace {

// layout of the scratch array (FP64 words)
constexpr int64_t SCR_VEC = TBDG_NOALLOC_MAX_NP;                 // one pressure vector
constexpr int64_t SCR_RED_PART = 64 * 4096;                       // reduction partials
constexpr int64_t SCR_RED_OUT = 128;                              // device scalars
constexpr int64_t SCR_RED_OP = TBDG_NOALLOC_MAX_NP + 1;           // operator-kernel partials
constexpr int64_t SCR_WORDS = 4 * SCR_VEC + SCR_RED_PART + SCR_RED_OUT + SCR_RED_OP;

__device__ __align__(256) double scratch[SCR_WORDS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

void noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) throw Error(TBDG_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return;
    int cur = -1;
    TBDG_HIP(hipGetDevice(&cur));
    if (cur != device) throw Error(TBDG_EDEVICE, "scratch set-up needs its device current");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        throw Error(TBDG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = static_cast<double*>(p);
}

NoallocScratch noalloc_scratch(int device) {
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (device >= 0 && device < MAX_DEVICES) base = g_ptr[device];
    }
    if (!base) {
        noalloc_init(device);
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_ptr[device];
    }
    NoallocScratch s;
    s.cr = base;
    s.cp = base + SCR_VEC;
    s.cq = base + 2 * SCR_VEC;
    s.cp2 = base + 3 * SCR_VEC;
    s.red_part = base + 4 * SCR_VEC;
    s.red_blocks = (int)SCR_RED_PART;
    s.red_out = s.red_part + SCR_RED_PART;
    s.red_op = s.red_out + SCR_RED_OUT;
    s.red_op_len = SCR_RED_OP;
    return s;
}

}  // namespace trbdg
