"""MI355X-native face transfer across 3:1 AMR resolution transitions."""
