"""CPU FP64 oracle (test infrastructure only; see sketchmp_oracle.py).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use this
package.  It never imports the product package and the product never imports it.
"""
from . import sketchmp_oracle  # noqa: F401
from .cmp import build_c_oracle, c_oracle  # noqa: F401
