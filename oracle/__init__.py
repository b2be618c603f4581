"""Plain FP64 CPU oracle for enforced-sparsity NMF.

TEST INFRASTRUCTURE ONLY.  It exists to check the HIP library, and only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The library never calls it and shares no code with it.
"""

from .als import (  # noqa: F401
    MODE_COLUMN,
    MODE_NONE,
    MODE_WHOLE,
    NotSPD,
    OracleState,
    als,
    clamp,
    error,
    error_direct,
    gram_dead,
    half_step,
    loss,
    loss_grad,
    residual,
    topt_per_column,
    topt_whole,
)
from .accuracy import topic_accuracy, alpha_beta  # noqa: F401
from .sequential import deflated_half_step, sequential_als  # noqa: F401
