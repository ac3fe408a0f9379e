// Test helper: rocRAND's own Philox4x32-10 block function (open-source
// header from the ROCm installation), exposed through a C entry point so the
// oracle's independently written Philox can be checked against it.  Built
// with g++ for the host only; nothing here is used by the GPU library.
#include <rocrand/rocrand_philox4x32_10.h>

struct open_engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

extern "C" void rr_philox(const unsigned* ctr, const unsigned* key, unsigned* out, int n)
{
    open_engine e;
    for (int i = 0; i < n; i++) {
        uint4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k = {key[2 * i], key[2 * i + 1]};
        uint4 r = e.ten_rounds(c, k);
        out[4 * i] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}
