// Stabilizer tableau (the STAB side of Table II) and its exact dense export.
//
// The tableau is the one of Aaronson and Gottesman (Phys. Rev. A 70,
// 052328, 2004): 2n rows of X bits, Z bits and a sign, rows 0..n-1 the
// destabilizers and n..2n-1 the stabilizer generators of the state; a row
// (x, z, r) stands for (-1)^r times the Pauli string with X where only x is
// set, Z where only z is, Y where both are. Clifford gates update every row
// by the paper's rules; the product of two rows ("rowsum") carries the sign
// through the per-qubit phase function g.
//
// Export (STAB -> SV, exact): the stabilizer rows are brought to reduced
// echelon form on their X bits (rows 0..r-1 with X pivots p_i, the others
// Z-type), a basis state x0 of the support is solved from the Z-type rows
// (z_j . x0 = r_j), and the state is 2^{-r/2} sum over c in GF(2)^r of
// (prod_{i: c_i = 1} g_i)|x0>, the expansion of prod_i (1 + g_i)/2 |x0>
// (the generators commute); its amplitude at x0 is real and positive.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/qw.h"
#include "qw_internal.h"

namespace qw {

namespace {

inline int popc(uint64_t v) { return __builtin_popcountll(v); }

// Phase exponent (powers of i) that qubit j contributes when row 1 (x1, z1)
// multiplies row 2 (x2, z2) from the left.
inline int g_phase(int x1, int z1, int x2, int z2) {
    if (!x1 && !z1) return 0;
    if (x1 && z1) return z2 - x2;
    if (x1) return z2 * (2 * x2 - 1);
    return x2 * (1 - 2 * z2);
}

}  // namespace

Tableau::Tableau(int n_) : n(n_), x(2 * n_, 0), z(2 * n_, 0), r(2 * n_, 0) {
    for (int i = 0; i < n; ++i) {
        x[i] = 1ull << i;      // destabilizer X_i
        z[n + i] = 1ull << i;  // stabilizer Z_i
    }
}

// Row h <- row i * row h (sign included).
void Tableau::rowsum(int h, int i) {
    int e = 2 * r[h] + 2 * r[i];
    for (int j = 0; j < n; ++j)
        e += g_phase((int)((x[i] >> j) & 1), (int)((z[i] >> j) & 1), (int)((x[h] >> j) & 1),
                     (int)((z[h] >> j) & 1));
    e = ((e % 4) + 4) % 4;
    r[h] = (uint8_t)(e == 2 ? 1 : 0);
    x[h] ^= x[i];
    z[h] ^= z[i];
}

void Tableau::h(int a) {
    for (int i = 0; i < 2 * n; ++i) {
        const uint64_t xa = (x[i] >> a) & 1, za = (z[i] >> a) & 1;
        r[i] ^= (uint8_t)(xa & za);
        x[i] = (x[i] & ~(1ull << a)) | (za << a);
        z[i] = (z[i] & ~(1ull << a)) | (xa << a);
    }
}

void Tableau::s(int a) {
    for (int i = 0; i < 2 * n; ++i) {
        const uint64_t xa = (x[i] >> a) & 1, za = (z[i] >> a) & 1;
        r[i] ^= (uint8_t)(xa & za);
        z[i] ^= xa << a;
    }
}

void Tableau::cx(int a, int b) {
    for (int i = 0; i < 2 * n; ++i) {
        const uint64_t xa = (x[i] >> a) & 1, za = (z[i] >> a) & 1;
        const uint64_t xb = (x[i] >> b) & 1, zb = (z[i] >> b) & 1;
        r[i] ^= (uint8_t)(xa & zb & (xb ^ za ^ 1));
        x[i] ^= xa << b;
        z[i] ^= zb << a;
    }
}

// Pauli gates flip the signs of the rows they anticommute with.
void Tableau::pauli(uint64_t px, uint64_t pz) {
    for (int i = 0; i < 2 * n; ++i) r[i] ^= (uint8_t)((popc(x[i] & pz) + popc(z[i] & px)) & 1);
}

std::string Tableau::apply(const qw_gate *g, uint64_t count) {
    for (uint64_t k = 0; k < count; ++k) {
        const qw_gate &q = g[k];
        char buf[128];
        const bool two = q.kind == QW_GATE_CNOT || q.kind == QW_GATE_CZ;
        if (q.q0 >= (uint32_t)n || (two && (q.q1 >= (uint32_t)n || q.q1 == q.q0)) || q.reserved) {
            snprintf(buf, sizeof buf, "gate %llu: bad qubits", (unsigned long long)k);
            return buf;
        }
        const int a = (int)q.q0, b = (int)q.q1;
        switch (q.kind) {
        case QW_GATE_X: pauli(1ull << a, 0); break;
        case QW_GATE_Z: pauli(0, 1ull << a); break;
        case QW_GATE_Y: pauli(1ull << a, 1ull << a); break;
        case QW_GATE_H: h(a); break;
        case QW_GATE_S: s(a); break;
        case QW_GATE_SDG: s(a); s(a); s(a); break;
        case QW_GATE_CNOT: cx(a, b); break;
        case QW_GATE_CZ: h(b); cx(a, b); h(b); break;
        default:
            snprintf(buf, sizeof buf, "gate %llu: kind 0x%x is not a Clifford gate of the tableau",
                     (unsigned long long)k, (unsigned)q.kind);
            return buf;
        }
    }
    return "";
}

StabExport Tableau::export_form() const {
    Tableau t = *this;
    const int S0 = n;  // stabilizer rows n..2n-1
    StabExport e;
    // reduced echelon form on the X bits
    int row = S0;
    for (int q = n - 1; q >= 0 && row < 2 * n; --q) {
        int piv = -1;
        for (int i = row; i < 2 * n; ++i)
            if ((t.x[i] >> q) & 1) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        if (piv != row) {
            std::swap(t.x[piv], t.x[row]);
            std::swap(t.z[piv], t.z[row]);
            std::swap(t.r[piv], t.r[row]);
        }
        for (int i = S0; i < 2 * n; ++i)
            if (i != row && ((t.x[i] >> q) & 1)) t.rowsum(i, row);
        e.pivot.push_back((uint32_t)q);
        ++row;
    }
    const int r_x = row - S0;
    // Z-type rows: reduced echelon form on the Z bits, then x0
    int zrow = row;
    std::vector<uint32_t> zpiv;
    for (int q = n - 1; q >= 0 && zrow < 2 * n; --q) {
        int piv = -1;
        for (int i = zrow; i < 2 * n; ++i)
            if ((t.z[i] >> q) & 1) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        if (piv != zrow) {
            std::swap(t.x[piv], t.x[zrow]);
            std::swap(t.z[piv], t.z[zrow]);
            std::swap(t.r[piv], t.r[zrow]);
        }
        for (int i = row; i < 2 * n; ++i)
            if (i != zrow && ((t.z[i] >> q) & 1)) t.rowsum(i, zrow);
        zpiv.push_back((uint32_t)q);
        ++zrow;
    }
    uint64_t x0 = 0;
    for (int j = row; j < zrow; ++j)
        if (t.r[j]) x0 |= 1ull << zpiv[(size_t)(j - row)];
    e.x0 = x0;
    for (int i = 0; i < r_x; ++i) {
        const int k = S0 + i;
        e.x.push_back(t.x[k]);
        e.z.push_back(t.z[k]);
        // powers of i of the row as i^{|x & z|} X^x Z^z, with its sign
        e.phase.push_back((uint8_t)((2 * t.r[k] + popc(t.x[k] & t.z[k])) & 3));
    }
    return e;
}

}  // namespace qw
