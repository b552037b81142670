// Host-side construction of Sobol' generator matrices (Sec. 2.3, Eq. ts).
//
// Primitive polynomials over F_2 are found by an order test: a polynomial p of degree d
// with p(0) = 1 is primitive iff x^(2^d - 1) = 1 mod p and x^((2^d - 1)/q) != 1 mod p for
// every prime q dividing 2^d - 1 (then x has order exactly 2^d - 1, which is only possible
// when the quotient ring is the field F_(2^d) and x generates its multiplicative group).
#include <cstdint>
#include <cstring>
#include <vector>

#include "qmc.h"

namespace qmc {
std::string& last_error_slot();
}

namespace {

// a * b mod p over F_2, with deg p = d <= 31 (operands below 2^d).
uint64_t gf2_mulmod(uint64_t a, uint64_t b, uint64_t p, int d) {
    uint64_t r = 0;
    for (int k = 0; k < d; ++k) {
        if ((b >> k) & 1u) r ^= a;
        a <<= 1;
        if ((a >> d) & 1u) a ^= p;
    }
    return r;
}

uint64_t gf2_powmod_x(uint64_t e, uint64_t p, int d) {
    uint64_t result = 1, base = 2 % p;
    if (d == 1) base = 2 ^ p;  // x mod (x + 1) = 1
    while (e) {
        if (e & 1u) result = gf2_mulmod(result, base, p, d);
        base = gf2_mulmod(base, base, p, d);
        e >>= 1;
    }
    return result;
}

std::vector<uint64_t> prime_factors(uint64_t n) {
    std::vector<uint64_t> f;
    for (uint64_t q = 2; q * q <= n; ++q) {
        if (n % q == 0) {
            f.push_back(q);
            while (n % q == 0) n /= q;
        }
    }
    if (n > 1) f.push_back(n);
    return f;
}

bool primitive(uint64_t p, int d) {
    if (d == 1) return p == 3;  // x + 1; the polynomial x is excluded
    if ((p & 1u) == 0) return false;
    const uint64_t order = (uint64_t(1) << d) - 1;
    if (gf2_powmod_x(order, p, d) != 1) return false;
    for (uint64_t q : prime_factors(order))
        if (gf2_powmod_x(order / q, p, d) == 1) return false;
    return true;
}

}  // namespace

extern "C" qmc_status qmc_primitive_polynomials(uint32_t count, uint32_t* codes) {
    if (count == 0) return QMC_OK;
    if (!codes) {
        qmc::last_error_slot() = "qmc_primitive_polynomials: codes is NULL";
        return QMC_ERR_INVALID_ARGUMENT;
    }
    if (count > 4096) {
        qmc::last_error_slot() = "qmc_primitive_polynomials: count above 4096";
        return QMC_ERR_OUT_OF_RANGE;
    }
    uint32_t found = 0;
    for (int d = 1; found < count && d <= 20; ++d) {
        for (uint64_t p = uint64_t(1) << d; p < (uint64_t(1) << (d + 1)) && found < count; ++p)
            if (primitive(p, d)) codes[found++] = static_cast<uint32_t>(p);
    }
    return QMC_OK;
}

extern "C" qmc_status qmc_sobol_matrices(uint32_t s, const uint32_t* direction_init, uint32_t* matrices) {
    return qmc_sobol_matrices_wide(s, direction_init, 32, matrices);
}

// Column k of a K-column matrix: the top 32 digits of the fraction m_(k+1) 2^-(k+1), i.e.
// m_(k+1) << (31 - k) below 32 and m_(k+1) >> (k - 31) from 32 on (m_(k+1) < 2^(k+1) <= 2^64).
extern "C" qmc_status qmc_sobol_matrices_wide(uint32_t s, const uint32_t* direction_init, uint32_t columns,
                                              uint32_t* matrices) {
    if (!direction_init || !matrices) {
        qmc::last_error_slot() = "qmc_sobol_matrices: NULL argument";
        return QMC_ERR_INVALID_ARGUMENT;
    }
    if (s == 0 || s > QMC_MAX_DIMS) {
        qmc::last_error_slot() = "qmc_sobol_matrices: s must be in [1, QMC_MAX_DIMS]";
        return QMC_ERR_OUT_OF_RANGE;
    }
    if (columns == 0 || columns > 64) {
        qmc::last_error_slot() = "qmc_sobol_matrices_wide: columns must be in [1, 64]";
        return QMC_ERR_OUT_OF_RANGE;
    }
    const int K = static_cast<int>(columns);
    std::vector<uint32_t> polys(s > 1 ? s - 1 : 1);
    if (s > 1) qmc_primitive_polynomials(s - 1, polys.data());

    // Dimension 0: identity, column k has only the 2^-(k+1) digit (none past 2^-32).
    for (int k = 0; k < K; ++k) matrices[k] = k < 32 ? 1u << (31 - k) : 0u;

    for (uint32_t j = 1; j < s; ++j) {
        const uint32_t p = polys[j - 1];
        int d = 31;
        while (!((p >> d) & 1u)) --d;
        if (d > QMC_MAX_DEGREE) {
            qmc::last_error_slot() = "qmc_sobol_matrices: polynomial degree above QMC_MAX_DEGREE";
            return QMC_ERR_OUT_OF_RANGE;
        }
        uint64_t m[64];
        const uint32_t* init = direction_init + size_t(j) * QMC_MAX_DEGREE;
        for (int k = 0; k < d; ++k) {
            m[k] = init[k];
            if ((m[k] & 1u) == 0 || m[k] >= (uint64_t(1) << (k + 1))) {
                qmc::last_error_slot() = "qmc_sobol_matrices: initial direction numbers must be odd and below 2^k";
                return QMC_ERR_INVALID_ARGUMENT;
            }
        }
        // Sobol' recurrence, in terms of the coefficient c_t of x^t (t = 1..d-1):
        //   m_k = m_(k-d) ^ (m_(k-d) << d) ^ XOR_t c_t (m_(k-d+t) << (d-t)).
        for (int k = d; k < K; ++k) {
            uint64_t v = m[k - d] ^ (m[k - d] << d);
            for (int t = 1; t < d; ++t)
                if ((p >> t) & 1u) v ^= m[k - d + t] << (d - t);
            m[k] = v;
        }
        for (int k = 0; k < K; ++k)
            matrices[size_t(j) * K + k] =
                static_cast<uint32_t>((k < 32 ? m[k] << (31 - k) : m[k] >> (k - 31)) & 0xFFFFFFFFu);
    }
    return QMC_OK;
}
