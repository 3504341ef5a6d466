// Operation-counting number type: executing a templated kernel body on the host
// with it counts the floating-point operations of one evaluation.
#pragma once

#include <cmath>

namespace gks {

struct OpCounts {
    long long add = 0, mul = 0, div = 0, transc = 0;
};

inline OpCounts &op_counts()
{
    static thread_local OpCounts c;
    return c;
}

struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
    explicit operator double() const { return v; }
};
static_assert(sizeof(Cnt) == 8, "Cnt must look like a double to the templates");

inline Cnt operator+(Cnt a, Cnt b) { ++op_counts().add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++op_counts().add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++op_counts().mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++op_counts().div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt &operator+=(Cnt &a, Cnt b) { a = a + b; return a; }
inline Cnt &operator-=(Cnt &a, Cnt b) { a = a - b; return a; }
inline Cnt &operator*=(Cnt &a, Cnt b) { a = a * b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }

template <>
__host__ __device__ inline Cnt erfc_t<Cnt>(Cnt x) { ++op_counts().transc; return Cnt(std::erfc(x.v)); }
template <>
__host__ __device__ inline Cnt exp_t<Cnt>(Cnt x) { ++op_counts().transc; return Cnt(std::exp(x.v)); }
template <>
__host__ __device__ inline Cnt expm1_t<Cnt>(Cnt x) { ++op_counts().transc; return Cnt(std::expm1(x.v)); }
template <>
__host__ __device__ inline Cnt pow_t<Cnt>(Cnt x, Cnt y) { ++op_counts().transc; return Cnt(std::pow(x.v, y.v)); }
template <>
__host__ __device__ inline Cnt sqrt_t<Cnt>(Cnt x) { ++op_counts().transc; return Cnt(std::sqrt(x.v)); }

}  // namespace gks
