"""Host check of the LDS index identity the register FFTs rely on.

Every Stockham pass of the loss kernels' FFTs (one-wave and multi-wave, N up
to 4,096, radices 16 then 2/4/8, in either pass order) addresses element r of
butterfly j at lds_pad(i + r S), lds_pad(i) = i + i // 16; the kernels write
this as a per-lane base lds_pad(i) plus a constant lds_off(r S).  This test
enumerates every (N, order, pass, butterfly, element) and checks that the two
agree, for the reads (i = j, S = N / R) and the writes (i = (j // Ns) Ns R +
j % Ns, S = Ns).
"""


def lds_pad(i):
    return i + (i >> 4)


def lds_off(ks):
    return ks + (ks >> 4)


def npass(logn):
    return logn // 4 + (1 if logn % 4 else 0)


def radix(logn, p):
    return 16 if p < logn // 4 else 1 << (logn % 4)


def test_lds_offsets_are_compile_time_constants():
    for logn in range(1, 13):
        n = 1 << logn
        passes = npass(logn)
        for order in (+1, -1):
            radices = [radix(logn, p if order > 0 else passes - 1 - p) for p in range(passes)]
            ns = 1
            for r_ in radices:
                b = n // r_
                for j in range(b):
                    d = (j // ns) * ns * r_ + j % ns
                    for r in range(r_):
                        assert lds_pad(j + r * b) == lds_pad(j) + lds_off(r * b)
                        assert lds_pad(d + r * ns) == lds_pad(d) + lds_off(r * ns)
                ns *= r_
            assert ns == n
