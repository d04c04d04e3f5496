"""Seeded synthetic inputs (tensors, legs, PEPOs) for the fPEPS row absorption.

Shared by the oracle, the tests and the benchmark. Holds no step of the
method itself: it only draws and stores data.
"""
from .tensor import Leg, Tensor, dense_tensor
from .configs import (Sym, Lattice, RowProblem, block_allowed, largest_remainder,
                      legs_dense, legs_u1u1, legs_su2, legs_u1u1_mini, legs_su2_mini, random_tensor, hubbard_pepo,
                      hubbard_pepo_site, hubbard_local_ops, identity_pepo, trivial_env,
                      random_top_env, random_peps, random_symmetric_pepo, config1_lattice,
                      config1_params, config2_row, random_bottom_env, config3_row, config4_row, small_row,
                      decaying_matrix, CONFIG5, su2_lattice, config4_lattice, lowrank_su2_lattice, LOWRANK_PARAMS, heff_inputs, bottom_closing, near_identity_pepo, KET_DIRS, PEPO_DIRS, ENV_DIRS)
