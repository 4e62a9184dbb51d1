"""Host-only parts of the density-matrix mode: the library's named Kraus operators against the
oracle's, and their argument errors (no GPU needed)."""
import numpy as np
import pytest

import paper_2211_07918_amd as Q
from oracle import density as Dm

KINDS = [(Q.QD_CHANNEL_DEPOLARIZING, Dm.depolarizing), (Q.QD_CHANNEL_DEPHASING, Dm.dephasing),
         (Q.QD_CHANNEL_AMPLITUDE_DAMPING, Dm.amplitude_damping)]


@pytest.mark.parametrize("kind,make", KINDS)
@pytest.mark.parametrize("d", [2, 3, 4, 5, 7])
@pytest.mark.parametrize("p", [0.0, 0.05, 0.5, 1.0])
def test_named_channels_match_the_oracle(kind, make, d, p):
    got = Q.qd_channel_kraus(kind, d, p)
    want = make(d, p)
    assert len(got) == len(want)
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(got, want)) <= 1e-15
    assert Dm.kraus_complete(got) <= 1e-14


def test_kraus_argument_errors():
    for args in ((7, 3, 0.1), (0, 1, 0.1), (0, 300, 0.1), (0, 3, -0.1), (0, 3, 1.5), (0, 3, float("nan"))):
        with pytest.raises(Q.QDError):
            Q.qd_channel_kraus(*args)
    out = np.zeros(9 * 9, dtype=np.complex128)
    n = Q.C.c_int32()
    rc = Q.load().qd_channel_kraus(0, 3, 0.1, out.ctypes.data_as(Q._DP), 2, Q.C.byref(n))
    assert rc == Q.QD_EINVAL and n.value == 9
