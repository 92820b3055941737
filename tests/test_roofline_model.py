"""The algorithmic byte and flop models bench.py divides by measured times, checked
against sizes derived by hand for the 128^3 Q1 hierarchy (levels as the setup builds
them) and against small cases counted block by block."""
import numpy as np

from paper_2606_24748_amd import roofline as RL

LEVELS = [{"nbr": 2146689, "bs": 3, "nnzb": 56638591, "p_nnzb": 9618228},
          {"nbr": 79507, "bs": 6, "nnzb": 2048383, "p_nnzb": 357911},
          {"nbr": 3375, "bs": 6, "nnzb": 79507, "p_nnzb": 12167},
          {"nbr": 125, "bs": 6, "nnzb": 2197, "p_nnzb": 0}]


def test_fine_spmv_bytes_hand_count():
    # 76 B per 3x3 FP64 block, int32 row pointers, x and y once
    want = 56638591 * 76 + 4 * (2146689 + 1) + 8 * (6440067 + 6440067)
    assert RL.spmv_bytes(2146689, 2146689, 3, 3, 56638591, 8, 8) == want == 4416160748


def test_spmv_bytes_brute_force_small():
    rng = np.random.default_rng(0)
    for br, bc, vs in ((3, 3, 8), (3, 6, 4), (6, 6, 2)):
        nbr, nbc, nnzb = int(rng.integers(1, 50)), int(rng.integers(1, 50)), int(rng.integers(0, 300))
        count = 0
        count += nnzb * (br * bc * vs)       # values
        count += nnzb * 4                    # column indices
        count += (nbr + 1) * 4               # row pointers
        count += nbc * bc * vs + nbr * br * vs  # x read, y written
        assert RL.spmv_bytes(nbr, nbc, br, bc, nnzb, vs, vs) == count


def test_pcg_iteration_bytes_128cube():
    fine = RL.spmv_bytes(2146689, 2146689, 3, 3, 56638591, 8, 8)
    f64 = RL.pcg_iteration_bytes(LEVELS, 8, 8)
    f32 = RL.pcg_iteration_bytes(LEVELS, 4, 4)
    # CG's FP64 product and its 10 vector passes are the same in both hierarchies
    common = fine + 10 * 8 * 6440067
    # the level-0 operator's four products dominate the hierarchy's share
    assert f64 - common > 4 * fine
    assert abs(f64 / 1e9 - 29.09) < 0.01 and abs(f32 / 1e9 - 17.55) < 0.01
    # an FP32 hierarchy halves the hierarchy's bytes (indices stay 4 B)
    assert (f32 - common) < 0.6 * (f64 - common)


def test_ptap_flops_per_pair():
    # 3x3 A block times 3x6 P block: 2*3*3*6 flops; 6x3 R block times 3x6 A P block: 2*6*3*6
    assert RL.ptap_flops(1, 0, 3, 6) == 108 and RL.ptap_flops(0, 1, 3, 6) == 216
    assert RL.ptap_flops(1, 1, 6, 6) == 2 * 6 * 6 * 6 * 2
