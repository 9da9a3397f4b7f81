"""Check of the breakdown decisions a GPU run hands to the oracle.

The parity tests replay the GPU's breakdown steps in the oracle
(force_breakdown), so both sides restart at the same steps with the same
vectors. A replayed step is only legitimate if the oracle, computing the same
step in FP64, also finds the new vector's norm negligible: at most `factor`
times the breakdown threshold of the GPU's working precision (100 unit
roundoffs times the largest bidiagonal entry so far). A GPU that broke down
where the true norm is sizeable fails here even though the replayed oracle
would follow it.
"""
import numpy as np

UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}


def check_replayed_breakdowns(ref, prec, factor=10.0):
    bd = 1e2 * UNIT_ROUNDOFF[prec]
    for side, j, val, scale in ref.get("forced", []):
        limit = factor * bd * scale
        assert val <= limit or val == 0.0, (
            f"replayed breakdown {side}{j}: oracle norm {val:.3e} exceeds {factor} x the "
            f"{prec} threshold ({limit:.3e}, scale {scale:.3e})")
    return len(ref.get("forced", []))
