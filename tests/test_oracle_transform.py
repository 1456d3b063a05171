"""Pins for the analytic spectrum and the Eq. 3 decomposition (Sec. II-F).

Analytic signal: brute-force DFT on tiny inputs, Re(analytic) = input, and the exact
analytic signal of a bin-centred cosine.  Decomposition: theta_o = 0 reduces to a plain
sum, integer advances reduce to circular shifts of the length-T' analytic traces, a
Gaussian-windowed tone moves by exactly the fractional advance, and a simulated point
scatterer appears where stationary phase puts it.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2603_22496_amd import configs as C
from paper_2603_22496_amd.phantom import Acquisition, Scatterers, make_dataset


def test_analytic_spectrum_matches_direct_dft():
    rng = np.random.default_rng(0)
    T, tp = 37, 64
    x = rng.integers(-300, 300, size=(2, T)).astype(np.int16)
    A = O.analytic_spectrum(x, tp)
    for r in range(2):
        for k in range(tp // 2 + 1):
            s = sum(float(x[r, n]) * complex(math.cos(-2 * math.pi * k * n / tp),
                                             math.sin(-2 * math.pi * k * n / tp)) for n in range(T))
            h = 1.0 if k in (0, tp // 2) else 2.0
            assert abs(A[r, k] - h * s) < 1e-9


def test_real_part_of_analytic_signal_is_the_record():
    rng = np.random.default_rng(1)
    x = rng.integers(-32768, 32767, size=(3, 5, 300)).astype(np.int16)
    a = O.analytic_signal(x, 512)
    assert np.max(np.abs(a.real - x)) < 1e-9
    assert np.max(np.abs(a.imag)) > 100.0


def test_analytic_signal_of_bin_centred_cosine():
    tp = 256
    n = np.arange(tp)
    for k0 in (1, 17, 100, 127):
        x = np.cos(2 * np.pi * k0 * n / tp)
        a = O.analytic_signal(x, tp)
        assert np.max(np.abs(a - np.exp(2j * np.pi * k0 * n / tp))) < 1e-12


def test_broadside_decomposition_is_plain_sum():
    ds = C.tiny_dataset(3)
    shift = np.zeros((1, ds.rf.shape[1]), dtype=np.int32)
    R = O.decompose(ds.rf, shift, 2048)
    a = O.analytic_signal(ds.rf, 2048)
    assert np.max(np.abs(R[:, 0, :] - a.sum(axis=1))) < 1e-8 * np.max(np.abs(R))


def test_integer_advances_are_circular_shifts():
    rng = np.random.default_rng(4)
    N, L, T, tp = 2, 6, 200, 256
    x = rng.integers(-2000, 2000, size=(N, L, T)).astype(np.int16)
    m = np.array([[0, 3, 7, 11, 40, 56], [5, 0, 1, 2, 3, 4]])
    R = O.decompose(x, (m << 22).astype(np.int32), tp)
    full = O.inverse_bins(O.analytic_spectrum(x, tp), tp, tp)     # length-T' analytic traces
    for i in range(N):
        for o in range(2):
            expect = sum(np.roll(full[i, l], -m[o, l])[:T] for l in range(L))
            assert np.max(np.abs(R[i, o] - expect)) < 1e-9 * np.max(np.abs(expect))


def test_fractional_advance_moves_a_band_limited_pulse():
    # x[n] = g(n - nc) cos(2 pi f (n - nc)); its analytic signal is g exp(i 2 pi f (n - nc))
    # to ~1e-19 at f = 0.25 cycles/sample, sigma = 6 samples.  An advance of s samples must
    # give g(n + s - nc) exp(i 2 pi f (n + s - nc)).
    T, tp, nc, sig, f = 300, 1024, 250.0, 6.0, 0.25
    n = np.arange(T)
    x = np.exp(-((n - nc) ** 2) / (2 * sig * sig)) * np.cos(2 * np.pi * f * (n - nc))
    for s in (0.37, 17.625, 100.0 + 1.0 / 3.0, 211.71):
        sq = int(round(s * 2 ** 22))
        sv = sq / 2 ** 22
        R = O.decompose(x[None, None, :], np.array([[sq]], dtype=np.int32), tp)[0, 0]
        m = n + sv - nc
        expect = np.exp(-(m ** 2) / (2 * sig * sig)) * np.exp(2j * np.pi * f * m)
        assert np.max(np.abs(R - expect)) < 1e-9, s


def test_point_scatterer_lands_where_stationary_phase_puts_it():
    # One scatterer, one broadside transmit.  Eq. 3 with edge references puts the echo at
    # t = z/c + [z cos(th_o) - (x - x_ref) sin(th_o)]/c  when the stationary element
    # u* = x + z tan(th_o) lies well inside the aperture.
    acq = Acquisition(L=128, T=2048, N=2, pitch=0.3e-3, c=1540.0, fs=20e6, fc=5e6,
                      theta_max=math.radians(1.0))
    xs, zs = 5e-3, 25e-3
    ds = make_dataset(acq, Scatterers.points([(xs, zs, 1.0)]))
    u = O.element_positions(128, 0.3e-3)
    rx = [math.radians(a) for a in (-8.0, -3.0, 0.0, 3.0, 8.0)]
    shift = np.array(O.luts.shear_table(128, 0.3e-3, 1540.0, 20e6, rx), dtype=np.int32)
    R = O.decompose(ds.rf, shift, 4096)
    th_i = acq.tx_angles()[0]
    for o, th in enumerate(rx):
        ustar = xs + zs * math.tan(th)
        assert u[0] + 3e-3 < ustar < u[-1] - 3e-3
        xref = u[0] if th >= 0 else u[-1]
        t = (xs * math.sin(th_i) + zs * math.cos(th_i)) / 1540.0 \
            + (zs * math.cos(th) - (xs - xref) * math.sin(th)) / 1540.0
        peak = int(np.argmax(np.abs(R[0, o])))
        assert abs(peak - t * 20e6) <= 1.0, (math.degrees(th), peak, t * 20e6)


def test_decomposition_is_linear():
    a, b = C.tiny_dataset(5), C.tiny_dataset(6)
    sh = np.array([[0, 1 << 22, 5 << 21, 123456789] * 4], dtype=np.int32)
    ra = O.decompose(a.rf, sh, 2048)
    rb = O.decompose(b.rf, sh, 2048)
    rab = O.decompose(a.rf.astype(np.int64) * 2 - b.rf.astype(np.int64), sh, 2048)
    assert np.max(np.abs(rab - (2 * ra - rb))) < 1e-9 * np.max(np.abs(rab))


def test_record_longer_than_fft_is_rejected():
    with pytest.raises(ValueError):
        O.analytic_spectrum(np.zeros((1, 300)), 256)


# ---------------------------------------------------------------------------------------
# Pins of decompose_spectrum (the per-bin contraction of Eq. 3 before the inverse transform)

def test_spectrum_is_the_transform_of_an_integer_shift_and_sum():
    # integer advances m_l: Eq. 3 is a time-domain shift-and-sum of the length-T' analytic
    # traces; its forward DFT must be the contraction output bin for bin (and zero above T'/2)
    rng = np.random.default_rng(11)
    N, L, T, tp = 2, 5, 90, 128
    x = rng.integers(-3000, 3000, size=(N, L, T)).astype(np.int16)
    m = np.array([[0, 1, 2, 3, 4], [9, 0, 17, 5, 33], [0, 0, 0, 0, 0]])
    Y = O.decompose_spectrum(x, (m << 22).astype(np.int32), tp)
    full = O.inverse_bins(O.analytic_spectrum(x, tp), tp, tp)
    for i in range(N):
        for o in range(m.shape[0]):
            y = sum(np.roll(full[i, l], -m[o, l]) for l in range(L))
            F = np.fft.fft(y)
            scale = np.max(np.abs(F))
            assert np.max(np.abs(Y[i, o] - F[: tp // 2 + 1])) < 1e-10 * scale
            assert np.max(np.abs(F[tp // 2 + 1:])) < 1e-10 * scale


def test_spectrum_of_bin_centred_cosine_under_fractional_advances():
    # x = cos(2 pi k0 n / T') over the whole record has one analytic bin, A[k0] = T'; an
    # advance of s samples multiplies it by exp(2 pi i k0 s / T'), summed over the elements
    tp, k0 = 256, 37
    n = np.arange(tp)
    L = 4
    x = np.tile(np.cos(2 * np.pi * k0 * n / tp), (1, L, 1))
    sq = np.array([[0, 1234567, -98765432, 2 ** 31 - 1], [5 << 22, (5 << 22) + 1, 7, -(1 << 30)]],
                  dtype=np.int64)
    Y = O.decompose_spectrum(x, sq.astype(np.int32), tp)
    for o in range(2):
        expect = sum(tp * complex(math.cos(2 * math.pi * k0 * (s / 2 ** 22) / tp),
                                  math.sin(2 * math.pi * k0 * (s / 2 ** 22) / tp)) for s in sq[o])
        assert abs(Y[0, o, k0] - expect) < 1e-9 * tp
        others = np.delete(Y[0, o], k0)
        assert np.max(np.abs(others)) < 1e-9 * tp


def test_spectrum_direct_dft_brute_force():
    # L = 4, N = 2, M = 3, T = 64: the analytic DFT of every record and the exactly reduced
    # phase turns evaluated bin by bin in plain Python
    rng = np.random.default_rng(12)
    N, L, M, T, tp = 2, 4, 3, 64, 128
    x = rng.integers(-32768, 32767, size=(N, L, T)).astype(np.int16)
    sh = rng.integers(-2 ** 31, 2 ** 31 - 1, size=(M, L)).astype(np.int32)
    Y = O.decompose_spectrum(x, sh, tp)
    period = tp << 22
    for i in range(N):
        for o in range(M):
            for k in range(tp // 2 + 1):
                h = 1.0 if k in (0, tp // 2) else 2.0
                acc = 0j
                for l in range(L):
                    a = sum(float(x[i, l, n]) * complex(math.cos(2 * math.pi * k * n / tp),
                                                        -math.sin(2 * math.pi * k * n / tp)) for n in range(T))
                    r = (k * int(sh[o, l])) % period
                    acc += h * a * complex(math.cos(2 * math.pi * r / period), math.sin(2 * math.pi * r / period))
                assert abs(Y[i, o, k] - acc) < 1e-7 * (1.0 + abs(acc)), (i, o, k)


def test_inverse_of_spectrum_is_the_decomposition():
    ds = C.tiny_dataset(2)
    rng = np.random.default_rng(13)
    sh = rng.integers(-2 ** 31, 2 ** 31 - 1, size=(3, ds.rf.shape[1])).astype(np.int32)
    Y = O.decompose_spectrum(ds.rf, sh, 2048)
    R = O.decompose(ds.rf, sh, 2048)
    assert np.max(np.abs(O.inverse_bins(Y, 2048, ds.rf.shape[2]) - R)) < 1e-12 * np.max(np.abs(R))
