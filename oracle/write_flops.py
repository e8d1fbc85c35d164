"""Write paper_2307_05683_amd/flops.py: algorithmic FP64 operations per
system-step, counted by running one step of the oracle's fixed-iteration
map (2 Halley steps with 4 series terms, 2 Newton steps with 8 terms,
combined drift, each planet pair once, combined jumps without GR) on an
operation-counting scalar type.  add/sub, mul, div and sqrt count one each
(an FMA counts as its multiply and its add)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2307_05683_amd", "flops.py")


def main():
    plain = {n: oracle.count_ops(n)["flops"] for n in range(1, 9)}
    gr = {n: oracle.count_ops(n, gr=True)["flops"] for n in range(1, 9)}
    # the integrator's second count set (wh_config.kepler_counts = 1): one
    # Halley step with 3 series terms, then 2 Newton steps with 8
    kc1 = {n: oracle.count_ops(n, n_halley=1, terms_halley=3)["flops"] for n in range(1, 9)}
    kc1_gr = {n: oracle.count_ops(n, gr=True, n_halley=1, terms_halley=3)["flops"] for n in range(1, 9)}
    jac = {n: oracle.count_ops_jacobi(n)["flops"] for n in range(1, 9)}
    jac_gr = {n: oracle.count_ops_jacobi(n, gr=True)["flops"] for n in range(1, 9)}
    with open(OUT, "w") as f:
        f.write('"""Algorithmic FP64 operations per system-step, by planet count.\n\n'
                'Counted on one step of the method as the paper states it (Sec. 3.1-3.4): the\n'
                'fixed-iteration Kepler solve of Sec. 3.2 (2 Halley steps with 4 series terms,\n'
                '2 Newton steps with 8), the combined drift, one evaluation per planet pair\n'
                '(third law, Sec. 3.3) and the jump(s).  add/sub, mul, div and sqrt count one\n'
                'each; an FMA counts two.  ALGO_FLOPS_JACOBI: the same drifts about the Jacobi\n'
                'Kepler masses and the closed-form Jacobi kick (no jump).  Written by\n'
                'oracle/write_flops.py.\n"""\n')
        f.write("ALGO_FLOPS = %r\n" % plain)
        f.write("ALGO_FLOPS_GR = %r\n" % gr)
        f.write("ALGO_FLOPS_JACOBI = %r\n" % jac)
        f.write("ALGO_FLOPS_JACOBI_GR = %r\n" % jac_gr)
        f.write("# kepler_counts = 1: one Halley step with 3 series terms, then 2 Newton steps with 8\n")
        f.write("ALGO_FLOPS_KC1 = %r\n" % kc1)
        f.write("ALGO_FLOPS_GR_KC1 = %r\n" % kc1_gr)
    print(OUT, plain, gr, jac, jac_gr)


if __name__ == "__main__":
    main()
