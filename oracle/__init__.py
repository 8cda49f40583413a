"""FP64 CPU oracle (test infrastructure only; see ``sgq_oracle``)."""
from .sgq_oracle import *  # noqa: F401,F403
from .sgq_oracle import BAND, FREE, GRAND  # noqa: F401
