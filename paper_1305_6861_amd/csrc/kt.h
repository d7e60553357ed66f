// Configuration populations of the K-t formalism (section 4.2), shared by
// the spin-spacing calculator (kt.cpp) and the K-t simulation engine
// (kt_engine.cpp).  Host code.
//
// When every gradient moment of a sequence is an integer multiple of a
// lattice step dk per axis, the magnetisation of a spin at x of one tissue
// is a finite series over lattice orders q (eq. 4.7 - 4.11),
//   Mxy(x) = sum_q F(q) exp(-2 pi j (q dk) . x),
//   Mz(x)  = sum_q Z(q) exp(-2 pi j (q dk) . x),
// whose populations depend on the RF pulses and the tissue's relaxation and
// off-resonance, never on x.  Hard pulses mix the triplet (F(q), conj F(-q),
// Z(q)) of each order with the complex form of eq. 3.19 (eq. 4.14),
// relaxation scales them and feeds Z(0) (eq. 4.15 / 4.16), a gradient of
// moment p dk moves every F(q) to q + p (eq. 4.17), and a spatially uniform
// off-resonance dw turns every F by exp(-j dw t).
#pragma once
#include <stdint.h>

#include <complex>
#include <unordered_map>

namespace ps {

using cplx = std::complex<double>;

// lattice order packed into 64 bits: 21 signed bits per axis
constexpr int64_t kKtBits = 21;
constexpr int64_t kKtLim = (int64_t(1) << (kKtBits - 1)) - 1;

int64_t kt_pack(int64_t a, int64_t b, int64_t c);
int64_t kt_axis(int64_t key, int d);
int64_t kt_negate(int64_t key);

struct KtTissue {
    double r1, r2;           // 1/T1, 1/T2 (0 for +inf)
    double dw = 0.0;         // rad/s, uniform over the tissue
};

// A gradient or a decay changes every transverse population in the same way
// (a shift of all orders by q, a factor e2 exp(-j dw tau)), so the store
// keeps them pending -- F(order) = stored F(order - shift) x scale -- and
// applies them only before a pulse mixes orders: stepping a readout sample
// by sample costs no rehashing.
class KtPopulations {
public:
    std::unordered_map<int64_t, cplx> Z;
    size_t peak = 0;         // most transverse configurations at once

    KtPopulations();
    void pulse(double alpha, double phi);
    void interval(double tau, const int64_t q[3], const KtTissue& t);
    void spoil();
    size_t n_transverse() const { return F_.size(); }
    // fn(packed order, population) for every transverse configuration
    template <typename Fn>
    void each_F(Fn&& fn) const {
        for (const auto& kv : F_)
            fn(kt_pack(kt_axis(kv.first, 0) + shift_[0], kt_axis(kv.first, 1) + shift_[1],
                       kt_axis(kv.first, 2) + shift_[2]),
               kv.second * scale_);
    }

private:
    std::unordered_map<int64_t, cplx> F_;
    int64_t shift_[3] = {0, 0, 0};
    cplx scale_ = 1.0;
    void settle();           // apply the pending shift and scale to the store
};

// The lattice vector q with m = q dk per axis (axes with dk = 0 carry no
// moment); false when m is off the lattice.
bool kt_lattice(const double m[3], const double dk[3], int64_t q[3]);

}  // namespace ps
