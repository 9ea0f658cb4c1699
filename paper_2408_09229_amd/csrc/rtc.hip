// Integrands compiled at run time (hipRTC): the counterpart of the paper's
// user-supplied integrand compiled for the GPU at run time (Sec. 3.6).
//
// The caller's source defines one device function,
//   __device__ vegas_real vegas_user_f(const vegas_real* x, int dim,
//                                      const double* params)
// and it is compiled together with the fill's own device headers into a
// fill kernel of its own: the same tile body (Alg. 2) as the built-in
// families, with the integrand's coordinates gathered into registers and
// passed to the caller's function at the end of the sample path.  The
// kernel is specialised to the problem's dimension (no per-axis guards).
// The headers travel inside the library (generated at build time), so
// nothing is read from disk at run time.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/vegas.h"
#include "host.hpp"
#include "layout.hpp"

// generated at build time from the device headers (build.py)
namespace vg_rtc_src {
extern const int kCount;
extern const char* const kNames[];
extern const char* const kTexts[];
}  // namespace vg_rtc_src

struct vegas_user_fn {
    int dim;
    int precision;
    int device;
    hipModule_t module;
    hipFunction_t fill;          // FP64 accumulators
    hipFunction_t fill_kahan;    // compensated FP32 accumulators (FP32 path only)
};

namespace vgh {

namespace {

std::string program_text(const char* user, int dim, bool fp64)
{
    std::string s;
    s += "#include \"fill_dev.hpp\"\n";
    s += fp64 ? "typedef double vegas_real;\n" : "typedef float vegas_real;\n";
    s += "#line 1 \"user integrand\"\n";
    s += user;
    s += "\n#line 1 \"vegas user fill\"\n";
    s += "namespace vg {\n"
         "template <> struct Fn<vegas_real, F_USER> {\n"
         "    const double* prm;\n"
         "    vegas_real xs[" + std::to_string(dim) + "];\n"
         "    __device__ __forceinline__ void setup(const SampleConst& sc, const vegas_real*) { prm = sc.prm; }\n"
         "    __device__ __forceinline__ void begin() {}\n"
         "    __device__ __forceinline__ void axis(int d, vegas_real x) { xs[d] = x; }\n"
         "    __device__ __forceinline__ vegas_real finish() const { return ::vegas_user_f(xs, " +
         std::to_string(dim) + ", prm); }\n"
         "};\n"
         "}  // namespace vg\n";
    const char* real = fp64 ? "double" : "float";
    for (int kahan = 0; kahan < (fp64 ? 1 : 2); ++kahan) {
        s += std::string("extern \"C\" __global__ __launch_bounds__(1024) void vegas_user_fill") +
             (kahan ? "_kahan" : "") + "(vg::FillArgs a)\n{\n"
             "    extern __shared__ __align__(16) unsigned char smem[];\n"
             "    vg::fill_body<" + real + ", vg::F_USER, " + std::to_string(dim) + ", " + (kahan ? "true" : "false") +
             ", true>(a, smem);\n}\n";
    }
    return s;
}

}  // namespace

int user_fn_dim(const vegas_user_fn* fn) { return fn->dim; }
int user_fn_precision(const vegas_user_fn* fn) { return fn->precision; }

hipError_t launch_user_fill(const vegas_user_fn* fn, const vg::FillArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    vg::FillArgs args = a;
    void* params[] = {&args};
    hipFunction_t f = a.accum == VEGAS_ACC_KAHAN ? fn->fill_kahan : fn->fill;
    return hipModuleLaunchKernel(f, n_wg, 1, 1, vg::kFillThreads, 1, 1, (unsigned)lds, st, params, nullptr);
}

}  // namespace vgh

using namespace vgh;

namespace {

vegas_status check_args(const char* source, int32_t dim, int32_t precision)
{
    if (!source) return fail(VEGAS_EINVAL, "null source");
    if (dim < 1 || dim > vg::kMaxDim) return fail(VEGAS_EINVAL, "dim must be 1..%d", vg::kMaxDim);
    if (precision != VEGAS_PREC_FP64 && precision != VEGAS_PREC_FP32)
        return fail(VEGAS_EINVAL, "unknown precision %d", precision);
    return VEGAS_OK;
}

// compile the user fill for one GPU architecture; code receives the code
// object
vegas_status rtc_compile(const char* source, int dim, bool fp64, const char* arch_name, std::vector<char>* code)
{
    const std::string text = program_text(source, dim, fp64);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, text.c_str(), "vegas_user.hip", vg_rtc_src::kCount, vg_rtc_src::kTexts,
                            vg_rtc_src::kNames) != HIPRTC_SUCCESS)
        return fail(VEGAS_EDEVICE, "hiprtcCreateProgram failed");
    const std::string arch = std::string("--gpu-architecture=") + arch_name;
    // the library's own flags: contraction off (the FP64 path's arithmetic
    // follows the written order), no packed FP32 instructions
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t log_n = 0;
    hiprtcGetProgramLogSize(prog, &log_n);
    std::string log(log_n, '\0');
    if (log_n) hiprtcGetProgramLog(prog, &log[0]);
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return fail(VEGAS_EINVAL, "the integrand did not compile: %s", log.c_str());
    }
    size_t code_n = 0;
    hiprtcGetCodeSize(prog, &code_n);
    code->resize(code_n);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return VEGAS_OK;
}

}  // namespace

extern "C" {

vegas_status vegas_user_check(const char* source, int32_t dim, int32_t precision)
{
    vegas_status s = check_args(source, dim, precision);
    if (s != VEGAS_OK) return s;
    std::vector<char> code;
    return rtc_compile(source, dim, precision == VEGAS_PREC_FP64, "gfx950", &code);
}

vegas_status vegas_user_compile(const char* source, int32_t dim, int32_t precision, vegas_user_fn** out)
{
    if (!out) return fail(VEGAS_EINVAL, "null out");
    *out = nullptr;
    vegas_status s = check_args(source, dim, precision);
    if (s != VEGAS_OK) return s;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    const bool fp64 = precision == VEGAS_PREC_FP64;
    std::vector<char> code;
    s = rtc_compile(source, dim, fp64, prop.gcnArchName, &code);
    if (s != VEGAS_OK) return s;
    vegas_user_fn* fn = new vegas_user_fn();
    fn->dim = dim;
    fn->precision = precision;
    fn->device = dev;
    fn->module = nullptr;
    fn->fill = fn->fill_kahan = nullptr;
    hipError_t e = hipModuleLoadData(&fn->module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&fn->fill, fn->module, "vegas_user_fill");
    if (e == hipSuccess && !fp64) e = hipModuleGetFunction(&fn->fill_kahan, fn->module, "vegas_user_fill_kahan");
    if (e != hipSuccess) {
        if (fn->module) (void)hipModuleUnload(fn->module);
        delete fn;
        return fail(VEGAS_EDEVICE, "loading the compiled integrand failed: %s", hipGetErrorString(e));
    }
    *out = fn;
    return VEGAS_OK;
}

void vegas_user_destroy(vegas_user_fn* fn)
{
    if (!fn) return;
    if (fn->module) (void)hipModuleUnload(fn->module);
    delete fn;
}

}  // extern "C"
