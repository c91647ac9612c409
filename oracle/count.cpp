// Counting build of the oracle -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY, like the oracle itself.
//
// The oracle's source (phx_oracle.c) compiled as C++ with every `double` replaced by a type that
// counts its arithmetic, per photon and per trace stage (sky: source, atmosphere, start plane;
// optics: entrance effects, obscuration, surfaces; sensor: silicon, diffusion, pixel), with the
// Philox blocks drawn and the screen bytes read.  The oracle marks its stages and pauses the
// count around arithmetic that is not the method's (decision margins kept for the tests,
// per-scene and per-device constants) and around the wavelength's position on the coating grid,
// which depends on the photon alone (its one subtraction and division per photon are left out
// rather than counted at every coated surface).  Counting conventions: an addition, subtraction or multiplication is one
// operation each (the oracle forms no fused multiply-adds: it is built without contraction);
// a division, a square root and a transcendental function (exp, log, sin, cos, tan, atan, pow
// with a non-integer exponent) one each in their own class; pow with a small integer exponent
// counts the multiplications of binary exponentiation; comparisons, negation, fabs and floor
// are not counted.  The layout of every struct is that of the oracle (the counting type holds
// one double), so a scene prepared by the oracle library can be traced here.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace orc_count {
enum { ADD, MUL, DIV, SQRT, TRANS, PHILOX, GATHER, N_FIELDS };
constexpr int N_STAGES = 3;
thread_local uint64_t tally[N_STAGES][N_FIELDS];
thread_local int stage = 0;
thread_local int paused = 0;
inline void bump(int f, uint64_t k = 1) {
    if (!paused) tally[stage][f] += k;
}
}  // namespace orc_count

struct cd {
    double v;
    cd() = default;
    template <class T, class = typename std::enable_if<std::is_arithmetic<T>::value>::type>
    cd(T x) : v((double)x) {}
    template <class T, class = typename std::enable_if<std::is_arithmetic<T>::value>::type>
    explicit operator T() const {
        return (T)v;
    }
    cd& operator+=(cd o) { orc_count::bump(orc_count::ADD); v += o.v; return *this; }
    cd& operator-=(cd o) { orc_count::bump(orc_count::ADD); v -= o.v; return *this; }
    cd& operator*=(cd o) { orc_count::bump(orc_count::MUL); v *= o.v; return *this; }
    cd& operator/=(cd o) { orc_count::bump(orc_count::DIV); v /= o.v; return *this; }
};
static_assert(sizeof(cd) == sizeof(double) && alignof(cd) == alignof(double), "layout");
static_assert(std::is_trivially_copyable<cd>::value, "trivially copyable");

inline cd operator+(cd a, cd b) { orc_count::bump(orc_count::ADD); return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { orc_count::bump(orc_count::ADD); return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { orc_count::bump(orc_count::MUL); return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { orc_count::bump(orc_count::DIV); return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline cd operator+(cd a) { return a; }
inline bool operator<(cd a, cd b) { return a.v < b.v; }
inline bool operator>(cd a, cd b) { return a.v > b.v; }
inline bool operator<=(cd a, cd b) { return a.v <= b.v; }
inline bool operator>=(cd a, cd b) { return a.v >= b.v; }
inline bool operator==(cd a, cd b) { return a.v == b.v; }
inline bool operator!=(cd a, cd b) { return a.v != b.v; }
inline bool operator!(cd a) { return !a.v; }

inline cd sqrt(cd a) { orc_count::bump(orc_count::SQRT); return cd(std::sqrt(a.v)); }
inline cd exp(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::exp(a.v)); }
inline cd log(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::log(a.v)); }
inline cd sin(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::sin(a.v)); }
inline cd cos(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::cos(a.v)); }
inline cd tan(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::tan(a.v)); }
inline cd atan(cd a) { orc_count::bump(orc_count::TRANS); return cd(std::atan(a.v)); }
inline cd pow(cd a, cd b) {
    const double e = b.v;
    if (e >= 1.0 && e <= 64.0 && e == std::floor(e)) {
        // binary exponentiation: squarings plus the extra multiplications of the set bits
        unsigned n = (unsigned)e, sq = 0, bits = 0;
        for (unsigned m = n; m > 1; m >>= 1) ++sq;
        for (unsigned m = n; m; m >>= 1) bits += m & 1u;
        orc_count::bump(orc_count::MUL, sq + bits - 1);
    } else {
        orc_count::bump(orc_count::TRANS);
    }
    return cd(std::pow(a.v, b.v));
}
inline cd floor(cd a) { return cd(std::floor(a.v)); }
inline cd fabs(cd a) { return cd(std::fabs(a.v)); }
inline bool isnan(cd a) { return std::isnan(a.v); }

#define ORC_STAGE(s) (orc_count::stage = (s))
#define ORC_COUNT_PAUSE() (++orc_count::paused)
#define ORC_COUNT_RESUME() (--orc_count::paused)
#define ORC_COUNT_PHILOX() orc_count::bump(orc_count::PHILOX)
#define ORC_COUNT_GATHER(bytes) orc_count::bump(orc_count::GATHER, (bytes))

#define double cd
extern "C" {
#include "phx_oracle.c"
}
#undef double

// The photons photon[0 .. count) of source src, as orc_trace_list, with counts[i][stage][field]
// the operations of photon i (fields: add/sub, mul, div, sqrt, transcendental, Philox blocks,
// screen bytes; stages: sky, optics, sensor).
extern "C" __attribute__((visibility("default"))) int orc_count_trace_list(
        const orc_scene* sc, int32_t src, const uint64_t* photon, uint64_t count,
        orc_event* events, uint64_t* counts) {
    if (src < 0 || src >= sc->n_src || (count && (!photon || !events || !counts))) return -1;
    for (uint64_t i = 0; i < count; ++i) {
        memset(orc_count::tally, 0, sizeof(orc_count::tally));
        orc_count::stage = 0;
        orc_count::paused = 0;
        trace_one(sc, src, photon[i], nullptr, &events[i]);
        memcpy(counts + i * orc_count::N_STAGES * orc_count::N_FIELDS, orc_count::tally,
               sizeof(orc_count::tally));
    }
    return 0;
}
