// CPU build of the library's FFT core (same source as the GPU kernels use), for
// checking codelets, Stockham index arithmetic and radix plans against numpy.
#include <cmath>
#include <vector>

#include "../../paper_1809_04195_amd/csrc/fft.hpp"

using namespace t2s;

template <int L>
static void run(int inv, int ntr, const float* in, float* out) {
    const int ld = lds_ld(L);
    std::vector<float2> a(ntr * ld), b(ntr * ld), tw(L);
    for (int m = 0; m < L; ++m) {
        const double ang = -2.0 * M_PI * m / L;
        tw[m] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
    }
    for (int t = 0; t < ntr; ++t)
        for (int i = 0; i < L; ++i) a[t * ld + ph(i)] = make_float2(in[2 * (t * L + i)], in[2 * (t * L + i) + 1]);
    float2* res = inv ? fft_emulate<L, true>(a.data(), b.data(), ntr, ld, tw.data())
                      : fft_emulate<L, false>(a.data(), b.data(), ntr, ld, tw.data());
    for (int t = 0; t < ntr; ++t)
        for (int i = 0; i < L; ++i) {
            out[2 * (t * L + i)] = res[t * ld + ph(i)].x;
            out[2 * (t * L + i) + 1] = res[t * ld + ph(i)].y;
        }
}

template <int R>
static void run_codelet(const float* in, float* out) {
    float2 v[R];
    for (int r = 0; r < R; ++r) v[r] = make_float2(in[2 * r], in[2 * r + 1]);
    dft<R>(v);
    for (int r = 0; r < R; ++r) {
        out[2 * r] = v[r].x;
        out[2 * r + 1] = v[r].y;
    }
}

extern "C" int fft_host(int L, int inv, int ntr, const float* in, float* out) {
    switch (L) {
        case 16: run<16>(inv, ntr, in, out); return 0;
        case 32: run<32>(inv, ntr, in, out); return 0;
        case 48: run<48>(inv, ntr, in, out); return 0;
        case 64: run<64>(inv, ntr, in, out); return 0;
        case 96: run<96>(inv, ntr, in, out); return 0;
        case 128: run<128>(inv, ntr, in, out); return 0;
        case 160: run<160>(inv, ntr, in, out); return 0;
        case 192: run<192>(inv, ntr, in, out); return 0;
        case 256: run<256>(inv, ntr, in, out); return 0;
        case 320: run<320>(inv, ntr, in, out); return 0;
        case 384: run<384>(inv, ntr, in, out); return 0;
        case 512: run<512>(inv, ntr, in, out); return 0;
    }
    return -1;
}

extern "C" int codelet_host(int R, const float* in, float* out) {
    switch (R) {
        case 2: run_codelet<2>(in, out); return 0;
        case 3: run_codelet<3>(in, out); return 0;
        case 4: run_codelet<4>(in, out); return 0;
        case 5: run_codelet<5>(in, out); return 0;
        case 6: run_codelet<6>(in, out); return 0;
        case 8: run_codelet<8>(in, out); return 0;
        case 10: run_codelet<10>(in, out); return 0;
        case 12: run_codelet<12>(in, out); return 0;
        case 16: run_codelet<16>(in, out); return 0;
        case 20: run_codelet<20>(in, out); return 0;
        case 24: run_codelet<24>(in, out); return 0;
        case 32: run_codelet<32>(in, out); return 0;
    }
    return -1;
}

extern "C" double root_re(long m, long n) { return root_of_unity(m, n).re; }
extern "C" double root_im(long m, long n) { return root_of_unity(m, n).im; }
