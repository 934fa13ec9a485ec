"""MI355X-native inverse fast multipole method (IFMM): HIP library + thin binding."""
from .ifmm import IFMM, IFMMError, factorize_batch, load_library  # noqa: F401
