"""Host-side schedule of pair symmetry (no GPU): the counters of plans that
transform unordered pairs.  The planner checks its round schedule itself
(every listed unordered pair once, no orbital twice in a round) and refuses
the plan otherwise, so a plan that builds has a valid schedule."""
import ctypes

import numpy as np
import pytest

from paper_1111_0716_amd import fock, inputs


def _stats(grid, kmesh, nb, prec=fock.FOCK_C64, kpairs=None, tuning=None):
    keep = []
    d = fock.make_desc(inputs.rhombohedral_lattice(9.56, 58.0), grid, inputs.gamma_mesh(*kmesh), None, nb, None,
                       0.106, kpairs, keep)
    h = ctypes.c_void_p()
    tn = fock.FockTuning(**tuning) if tuning else None
    st = fock.lib().fock_plan_tuned((fock.FockDesc * 1)(d), 1, prec, None, ctypes.byref(tn) if tn else None,
                                    ctypes.byref(h))
    assert st == fock.FOCK_OK, fock.lib().fock_last_error().decode()
    a, b, c, e = (ctypes.c_int64() for _ in range(4))
    fock.lib().fock_plan_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(e))
    fock.lib().fock_destroy(h)
    return a.value, b.value, e.value


@pytest.mark.parametrize("kmesh,nb", [((1, 1, 1), 1), ((1, 1, 1), 2), ((3, 1, 1), 5), ((2, 2, 2), 7),
                                      ((4, 4, 4), 18)])
def test_whole_pair_rounds_transform_each_unordered_pair_once(kmesh, nb):
    nk = int(np.prod(kmesh))
    o = nk * nb
    ordered, fft, launches = _stats((32, 32, 32), kmesh, nb, tuning={"fused_rounds": 1})
    assert ordered == o * o
    assert fft == o * (o + 1) // 2
    # one zero fill, then rounds of at most 512 disjoint pairs (at least ceil(o/2) rounds hold the o self pairs
    # and the perfect matchings)
    assert launches - 1 >= -(-fft // 512)
    o_ord, o_fft, _ = _stats((32, 32, 32), kmesh, nb, tuning={"no_pair_symmetry": 1})
    assert o_ord == ordered and o_fft == ordered


def test_32cubed_fp32_full_sets_take_the_symmetric_three_pass_path():
    """32^3 FP32 with the full k-pair set: three-pass batches of unordered
    pairs (fewer transforms than ordered pairs, three or four launches per
    batch); FP64 16^3 and FP32 24^3 stay on the whole-pair kernel."""
    ordered, fft, launches = _stats((32, 32, 32), (2, 2, 2), 18)
    assert fft < ordered and launches >= 3
    o2, f2, l2 = _stats((32, 32, 32), (2, 2, 2), 18, tuning={"no_pair_symmetry": 1})
    assert f2 == o2 and l2 <= 2
    o3, f3, l3 = _stats((24, 24, 24), (2, 2, 2), 18)
    assert f3 == o3 and l3 <= 2


def test_rounds_follow_an_explicit_symmetric_k_pair_list():
    kp = [[0, 0], [0, 1], [1, 0], [2, 3], [3, 2], [1, 1]]
    ordered, fft, _ = _stats((32, 32, 32), (2, 2, 1), 3, kpairs=kp, tuning={"fused_rounds": 1})
    assert ordered == len(kp) * 9
    # unordered: (0,0) and (1,1) 6 each with self pairs, (0,1) and (2,3) 9 each
    assert fft == 6 + 6 + 9 + 9


def test_three_pass_blocks_transform_fewer_pairs():
    ordered, fft, launches = _stats((72, 72, 72), (2, 2, 2), 160)
    assert ordered == 1_638_400
    o = 1280
    assert fft == o * (o + 1) // 2  # off-diagonal block pairs and triangular diagonal blocks
    _, fft_ord, _ = _stats((72, 72, 72), (2, 2, 2), 160, tuning={"no_pair_symmetry": 1})
    assert fft_ord == ordered


def test_asymmetric_lists_keep_ordered_pairs():
    kp = [[0, 1], [1, 1]]  # (1, 0) not listed
    ordered, fft, _ = _stats((32, 32, 32), (2, 1, 1), 3, kpairs=kp, tuning={"fused_rounds": 1})
    assert fft == ordered == 2 * 9
