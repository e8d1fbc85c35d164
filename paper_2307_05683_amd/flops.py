"""Algorithmic FP64 operations per system-step, by planet count.

Counted on one step of the method as the paper states it (Sec. 3.1-3.4): the
fixed-iteration Kepler solve of Sec. 3.2 (2 Halley steps with 4 series terms,
2 Newton steps with 8), the combined drift, one evaluation per planet pair
(third law, Sec. 3.3) and the jump(s).  add/sub, mul, div and sqrt count one
each; an FMA counts two.  ALGO_FLOPS_JACOBI: the same drifts about the Jacobi
Kepler masses and the closed-form Jacobi kick (no jump).  Written by
oracle/write_flops.py.
"""
ALGO_FLOPS = {1: 275, 2: 574, 3: 898, 4: 1247, 5: 1621, 6: 2020, 7: 2444, 8: 2893}
ALGO_FLOPS_GR = {1: 310, 2: 637, 3: 989, 4: 1366, 5: 1768, 6: 2195, 7: 2647, 8: 3124}
ALGO_FLOPS_JACOBI = {1: 329, 2: 683, 3: 1062, 4: 1466, 5: 1895, 6: 2349, 7: 2828, 8: 3332}
ALGO_FLOPS_JACOBI_GR = {1: 361, 2: 747, 3: 1158, 4: 1594, 5: 2055, 6: 2541, 7: 3052, 8: 3588}
# kepler_counts = 1: one Halley step with 3 series terms, then 2 Newton steps with 8
ALGO_FLOPS_KC1 = {1: 228, 2: 480, 3: 757, 4: 1059, 5: 1386, 6: 1738, 7: 2115, 8: 2517}
ALGO_FLOPS_GR_KC1 = {1: 263, 2: 543, 3: 848, 4: 1178, 5: 1533, 6: 1913, 7: 2318, 8: 2748}
