"""CPU FP64 oracle of the FDAS correlation hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import, call, link or execute anything under ``oracle/``.  The product
library (``paper_1511_07343_amd``) never imports it, and it never imports the
product library: the two share no code.  The only shared module is ``synth``,
which generates seeded inputs and holds none of the method's arithmetic.
"""
from .fdas_oracle import *  # noqa: F401,F403
from .fdas_oracle import __all__  # noqa: F401
