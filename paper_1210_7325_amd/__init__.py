"""MI355X-native solver for sequences of generalized least-squares problems."""
