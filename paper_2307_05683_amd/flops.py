"""Algorithmic FP64 operations per system-step, by planet count.

Counted on one step of the method as the paper states it (Sec. 3.1-3.4): the
fixed-iteration Kepler solve of Sec. 3.2 (2 Halley steps with 4 series terms,
2 Newton steps with 8), the combined drift, one evaluation per planet pair
(third law, Sec. 3.3) and the jump(s).  add/sub, mul, div and sqrt count one
each; an FMA counts two.  Written by oracle/write_flops.py.
"""
ALGO_FLOPS = {1: 313, 2: 650, 3: 1012, 4: 1399, 5: 1811, 6: 2248, 7: 2710, 8: 3197}
ALGO_FLOPS_GR = {1: 348, 2: 713, 3: 1103, 4: 1518, 5: 1958, 6: 2423, 7: 2913, 8: 3428}
