// Floating-point operation count of the oracle (TEST AND MEASUREMENT INFRASTRUCTURE ONLY).
//
// The oracle's own source (nsa_oracle.c, unchanged) is compiled here as C++ with `double` standing for
// a value type that counts every arithmetic operation it takes part in: +, -, *, / and sqrt / cbrt each
// count one (a fused multiply-add does not occur: the oracle is built without contraction), fabs, negation,
// comparisons and copies count none. Running the oracle's element loop over a mesh then gives the
// floating-point operations the method performs per element in the order of Listing 1 (Gauss-point
// loops included), the figure the paper's Table 1 reports for its own code. The counting build computes
// the same values as the plain oracle (checked by the tests).
//
// Build: g++ -O1 -ffp-contract=off -std=c++17 -fpermissive -fPIC -shared -o liboracle_flops.so flops.cpp
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace flopcount {

long long counter = 0;

struct fd {
    double v;
    fd() = default;
    fd(double x) : v(x) {}
    fd &operator+=(fd b) { counter++; v += b.v; return *this; }
    fd &operator-=(fd b) { counter++; v -= b.v; return *this; }
    fd &operator*=(fd b) { counter++; v *= b.v; return *this; }
    fd &operator/=(fd b) { counter++; v /= b.v; return *this; }
};
static_assert(sizeof(fd) == sizeof(double), "fd is a plain double in memory");

inline fd operator+(fd a, fd b) { counter++; return fd(a.v + b.v); }
inline fd operator-(fd a, fd b) { counter++; return fd(a.v - b.v); }
inline fd operator*(fd a, fd b) { counter++; return fd(a.v * b.v); }
inline fd operator/(fd a, fd b) { counter++; return fd(a.v / b.v); }
inline fd operator-(fd a) { return fd(-a.v); }
inline bool operator<(fd a, fd b) { return a.v < b.v; }
inline bool operator>(fd a, fd b) { return a.v > b.v; }
inline bool operator<=(fd a, fd b) { return a.v <= b.v; }
inline bool operator>=(fd a, fd b) { return a.v >= b.v; }
inline bool operator==(fd a, fd b) { return a.v == b.v; }
inline bool operator!=(fd a, fd b) { return a.v != b.v; }
inline bool operator!(fd a) { return !a.v; }
inline fd sqrt(fd a) { counter++; return fd(std::sqrt(a.v)); }
inline fd cbrt(fd a) { counter++; return fd(std::cbrt(a.v)); }
inline fd fabs(fd a) { return fd(std::fabs(a.v)); }
inline bool isfinite(fd a) { return std::isfinite(a.v); }

}  // namespace flopcount

using flopcount::cbrt;
using flopcount::fabs;
using flopcount::sqrt;

#define double flopcount::fd
#include "nsa_oracle.c"
#undef double

extern "C" {

// Operations of oracle_residual / oracle_assemble over the mesh (the scatter's adds included),
// returned with the status in *status.
long long oracle_flops_residual(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                                const double *veloc, double rho, double mu, double dt, double *rhsid, double *dt_rho,
                                double *mass_rho, int *status)
{
    flopcount::counter = 0;
    *status = oracle_residual(npoin, nelem, lnods, reinterpret_cast<const flopcount::fd *>(coord),
                              reinterpret_cast<const flopcount::fd *>(veloc), rho, mu, dt,
                              reinterpret_cast<flopcount::fd *>(rhsid), reinterpret_cast<flopcount::fd *>(dt_rho),
                              reinterpret_cast<flopcount::fd *>(mass_rho));
    return flopcount::counter;
}

long long oracle_flops_assemble(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                                const double *veloc, double rho, double mu, double dt, int64_t nnzb,
                                const int32_t *emap, double *values, double *rhs, int *status)
{
    flopcount::counter = 0;
    *status = oracle_assemble(npoin, nelem, lnods, reinterpret_cast<const flopcount::fd *>(coord),
                              reinterpret_cast<const flopcount::fd *>(veloc), rho, mu, dt, nnzb, emap,
                              reinterpret_cast<flopcount::fd *>(values), reinterpret_cast<flopcount::fd *>(rhs));
    return flopcount::counter;
}

}  // extern "C"
