// Host-only driver for the sanitizer test of the C ABI's argument validation.
//
// tests/test_sanitizers.py compiles the library's API translation unit with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side only, links
// it with the other objects, and runs this program on the CPU (no GPU is needed:
// every call below is rejected by host validation before any launch or device
// query).  Exit status 0 means every call returned the documented error code
// and no sanitizer report was raised.
#include <cstdint>
#include <cstdio>

#include "blocktransform.h"

static int failures = 0;

static void expect(const char *what, int got, int want)
{
    if (got != want) {
        std::fprintf(stderr, "%s: got %d, want %d\n", what, got, want);
        ++failures;
    }
}

int main()
{
    void *a = reinterpret_cast<void *>(uintptr_t(1) << 20);
    float *t = reinterpret_cast<float *>(uintptr_t(1) << 32);
    void *b = reinterpret_cast<void *>(uintptr_t(1) << 34);
    void *mis = reinterpret_cast<void *>((uintptr_t(1) << 20) + 4);
    for (int compute : {TF_FP32, TF_PLAIN_FP32, TF_SPLIT_BF16, TF_SPLIT_FP16}) {
        const int K = 1024, M = 15;
        expect("negative count", transform_forward(a, t, b, -1, K, M, 0, compute, nullptr, 0, nullptr), TF_EINVAL);
        expect("null input", transform_forward(nullptr, t, b, 4, K, M, 0, compute, nullptr, 0, nullptr), TF_EINVAL);
        expect("tap stride", transform_forward(a, t, b, 4, K, M, 7, compute, nullptr, 0, nullptr), TF_EINVAL);
        expect("misaligned", transform_forward(mis, t, b, 4, K, M, 0, compute, nullptr, 0, nullptr), TF_EINVAL);
        expect("in place", transform_forward(a, t, a, 4, K, M, 0, compute, nullptr, 0, nullptr), TF_EINVAL);
        expect("bad K", transform_forward(a, t, b, 4, 3, M, 0, compute, nullptr, 0, nullptr), TF_EUNSUPPORTED);
        expect("bad M", transform_forward(a, t, b, 4, K, 17, 0, compute, nullptr, 0, nullptr), TF_EUNSUPPORTED);
        expect("empty", transform_forward(nullptr, nullptr, nullptr, 0, K, M, 0, compute, nullptr, 0, nullptr), TF_OK);
        expect("inverse in place", transform_inverse(a, t, a, 4, K, M, 0, compute, nullptr, nullptr, 0, nullptr),
               TF_EINVAL);
        expect("adjoint tap gradient without S",
               transform_adjoint(a, t, nullptr, b, t, 4, K, M, 0, compute, nullptr, 0, nullptr), TF_EINVAL);
    }
    expect("unknown compute", transform_forward(a, t, b, 4, 16, 5, 0, 9, nullptr, 0, nullptr), TF_EUNSUPPORTED);
    expect("noalloc in place", transform_adjoint_noalloc(a, t, nullptr, a, nullptr, 4, 16, 5, 0, nullptr), TF_EINVAL);
    expect("noalloc bad K", transform_adjoint_noalloc(a, t, nullptr, b, nullptr, 4, 12, 5, 0, nullptr),
           TF_EUNSUPPORTED);
    tf_ragged_plan plan = nullptr;
    const int32_t Ks[2] = {48, 64}, Ms[2] = {3, 3};
    const int64_t off[2] = {0, 144};
    expect("ragged bad K", transform_ragged_plan_create(Ks, Ms, off, off, 2, 336, &plan), TF_EUNSUPPORTED);
    expect("ragged null plan", transform_ragged_plan_create(Ks, Ms, off, off, 2, 336, nullptr), TF_EINVAL);
    expect("ragged negative", transform_ragged_plan_create(Ks, Ms, off, off, -1, 336, &plan), TF_EINVAL);
    expect("ragged execute null", transform_ragged_execute(nullptr, 0, a, t, b, nullptr, nullptr, nullptr, 0, nullptr),
           TF_EINVAL);
    for (int s : {0, -1, -2, -3, -4, -5, 7}) {
        const char *txt = transform_status_string(s);
        if (!txt || !txt[0]) ++failures;
    }
    std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
